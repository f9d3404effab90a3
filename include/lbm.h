/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the EOS-based multiphase
 * lattice Boltzmann method of He, Qin, Chen & Wen, "Numerical simulation of
 * pulmonary airway reopening by the EOS-based multiphase lattice Boltzmann
 * method" (arXiv 2103.08301).
 *
 * One call of lbm_step advances a D2Q9 lattice by n time steps.  Each step is
 * one fused HIP kernel that
 *   - pull-streams the post-collision distributions (left side of eq. 2.1),
 *     with halfway bounce-back at the walls and extrapolated or periodic ends
 *     (Sec. 2.3, airway model),
 *   - forms the density and the EOS field phi = k^2 p0(rho) - rho c_s^2
 *     (eqs. 2.12, 2.17, 2.18), with wetting ghost rows of density rho_wall,
 *   - evaluates the nonideal force F = -grad phi + kappa rho grad(lap rho)
 *     (eq. 2.17) plus the pressure-drop body force dp/nx along +x,
 *   - applies the velocity-shift forcing u_eq = u + tau F/rho and
 *     v = u + F/(2 rho) (Sec. 2.2, last paragraph before "Verification"),
 *   - relaxes in moment space with the MRT operator of eq. 2.1 and the rates
 *     printed after it, and stores the new distributions,
 *   - and, on the two first fluid rows next to each wall, produces the wall
 *     shear stress and wall pressure (Figs. 3, 5, 8 of the paper) with FP64
 *     per-step extremes and time integrals.
 *
 * Conventions
 *   - Every call returns lbm_status: 0 on success, a negative code otherwise;
 *     lbm_last_error(ctx) then holds a message.  A call that fails with
 *     LBM_EINVAL has no side effects.
 *   - Host arrays are caller-owned, row-major [ny][nx] with x fastest;
 *     distributions are [9][ny][nx] in the D2Q9 order
 *       e0=(0,0) e1=(1,0) e2=(0,1) e3=(-1,0) e4=(0,-1)
 *       e5=(1,1) e6=(-1,1) e7=(-1,-1) e8=(1,-1).
 *   - Device memory is caller-owned: the caller allocates lbm_workspace()
 *     bytes (any allocator; 256-byte alignment) and binds it with lbm_bind()
 *     together with the HIP stream on which every kernel is launched.  The
 *     library itself never allocates device memory.
 *   - Walls lie at y = -1/2 and y = ny - 1/2 (channel width ny); cell centres
 *     are at integer (x, y).
 *   - A context is not thread-safe; separate contexts are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument; nothing was changed */
    LBM_ENOMEM = -2,     /* host allocation failed, or the bound workspace is too small */
    LBM_EDEVICE = -3,    /* a HIP call failed; the message names it */
    LBM_EUNSTABLE = -4,  /* a stability check found NaN or |v| > v_limit; see lbm_check_state */
    LBM_ESTATE = -5      /* call out of order (e.g. lbm_step before lbm_bind / lbm_init_*) */
} lbm_status;

typedef enum { LBM_EOS_CS = 0, LBM_EOS_PR = 1 } lbm_eos_kind;

/* Storage of the distributions in device memory and arithmetic of the step:
   F64: FP64 / FP64.  F32: FP32 / FP32, with the EOS field phi of eq. 2.17 and
   its gradient in FP64.  F16S, BF16S: f_i - 9 w_i q in FP16 / BF16, FP32
   arithmetic on those deviations (q: see rho0_shift).  F32D: FP32 storage, FP64
   arithmetic.  F32S: f_i - 9 w_i q in FP32, FP32 arithmetic on the deviations,
   phi in FP64. */
/* Storage of the distributions.  F64T keeps each population as an FP64 value
   and its FP64 tangent along a direction of the parameters (lbm_set_tangent):
   the step then runs in tangent-linear arithmetic and the wall summaries carry
   the derivative of the squared wall shear (forward-mode sensitivities).  F64T
   runs on the tile schedule with 12-row, 8-wave tiles, CS or PR.
   F16R: f_i - 9 w_i q in FP16 with stochastic rounding, FP32
   arithmetic: each stored value rounds up or down to a neighbouring FP16 value
   with probabilities that make the expected rounding error zero, the random
   bits coming from an integer hash of (step counter, node, direction), so runs
   are reproducible.  Round-to-nearest FP16 storage (F16S) repeats the same
   error every step where the populations are steady, which acts as a mass
   source; F16R averages it out.  Tile schedule (one step per launch) and
   batches; no adjoint. */
typedef enum {
    LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3, LBM_F32D = 4, LBM_F32S = 5, LBM_F64T = 6, LBM_F16R = 7
} lbm_storage;

typedef struct {
    int eos;             /* lbm_eos_kind. CS: Carnahan-Starling p0 = rho R T (1+h+h^2-h^3)/(1-h)^3 - a rho^2,
                            h = b rho/4.  PR: eq. 2.18 with the standard alpha(T). */
    double a, b, R;      /* EOS constants (CS: 1, 4, 1; PR in the paper: 2/49, 2/21, 1) */
    double omega;        /* PR acentric factor (paper: 0.344 water, 0.011 methane) */
    double T_over_Tc;    /* temperature as a fraction of the EOS critical temperature,
                            which the library solves from (a, b, R) */
    double k;            /* proportional coefficient of eqs. 2.13-2.17 (mesh units: phi = k^2 p0 - rho/3) */
    double kappa;        /* gradient coefficient of eq. 2.17 (paper: 0.001) */
    double s_e, s_eps, s_q;  /* MRT rates (paper: 1.64, 1.54, 1.7); s_v = 1/tau */
    double s_j;          /* momentum-row rate; <= 0 selects 1/tau (so the velocity shift adds exactly F) */
    double rho_wall;     /* virtual density of the wall ghost rows (wettability); NaN selects rho_l(T) */
    double dp;           /* pressure drop along +x; uniform body force density dp/nx */
    int x_periodic;      /* 1: periodic ends; 0: extrapolated (zero-gradient) ends */
    int y_periodic;      /* 1: no walls, periodic in y (test mode; no wall diagnostics) */
    int storage;         /* lbm_storage */
    double rho0_shift;   /* density shift rho0 of the shifted storages (F32S, F16S, F16R, BF16S);
                            NaN selects rho_g(T).  They store f_i - 9 w_i q with q = rho0 / 9
                            rounded to a multiple of 2^-24, so that the shift constants
                            9 w_i q (w_i = 4/9, 1/9, 1/36) have few bits and an FP16 value
                            plus its shift is exact in FP32 (below 1/4) */
    int check_every;     /* stability/interface check cadence in steps (>= 1) */
    double v_limit;      /* a check fails when |v| exceeds this or a NaN appears */
    int history_cap;     /* capacity (steps) of the device ring of per-step wall summaries (>= 1) */
    int tile_rows;       /* output rows per tile or per wave chunk; 0 selects the default.
                            schedule 0: 8, 12, 20 or 28 (default 8, or 12 with FP64 arithmetic or 8 waves);
                            schedule 1: 4..256 (default 16);
                            schedule 2: 4, 8 or 12 with 4 waves, 8 or 16 with 8 waves (default 8) */
    int schedule;        /* 0: one block per 60 x tile_rows tile, phases coupled through LDS;
                            1: one wavefront per 60-column strip marching up a row chunk;
                            2: the tiles of schedule 0 taken one after another by resident blocks
                               (per-XCD ticket counters in the workspace), the next tile's loads
                               issued before the current tile is computed */
    int tile_waves;      /* schedules 0 and 2: waves per tile block, 0 (= 4), 4 or 8; schedule 1: 0 */
    int pipe_blocks;     /* schedule 2: blocks launched; 0 = compute units x blocks one unit holds,
                            otherwise >= 8 (every one of the 8 tile ranges needs a block) */
    int graph_steps;     /* schedules 0 and 1 (and batches): steps per captured HIP graph of step launches,
                            replayed instead of launching kernel by kernel; 0 selects 64, -1 launches every
                            step directly; otherwise 2, 4, 8, 16, 32, 64, 128 or 256 */
    int fused_steps;     /* schedule 0 (single lattices and batches, not F64T or F16R): steps per launch, 0
                            (= 1), 1 or 2.  2: one launch advances two steps, keeping the intermediate
                            populations in LDS (54 x 14-row tiles, 54 x 6 with FP64 arithmetic), bit-identical to
                            two one-step launches; it halves the HBM traffic per step, which pays when the
                            distributions do not fit the Infinity Cache, while on smaller lattices the longer tile
                            chain's latency makes it slower, so it is not the default (lbm_autotune times both).
                            The step that emits fields, and the last step of a call, are one-step launches */
} lbm_params;

/* Per-step wall summary ([0] bottom wall, [1] top wall).  FP64. */
typedef struct {
    int64_t step;                        /* 1-based index of the step */
    double tau_max[2], tau_min[2];       /* wall shear stress extremes over x */
    double p_max[2], p_min[2];           /* wall pressure extremes over x */
    int32_t x_tau_max[2], x_tau_min[2];  /* smallest x attaining each extreme */
    int32_t x_p_max[2], x_p_min[2];
    double sum_tau2;                     /* sum over both walls and all x of tau_w^2 */
    double int_peak_tau2;                /* running sum over steps of max over walls and x of tau_w^2 */
    double int_tau2;                     /* running sum over steps of sum_tau2 */
    double run_tau_max[2], run_tau_min[2];  /* extremes over x and over steps 1..step since the
                                               initialisation: run_*_max - run_*_min is the span of
                                               wall stress over a rupture (Sec. 3.2-3.3) */
    double run_p_max[2], run_p_min[2];
    double d_sum_tau2;                   /* F64T storage: derivative of sum_tau2 along the tangent direction */
    double d_int_tau2;                   /* F64T storage: derivative of int_tau2 along the tangent direction */
} lbm_stress_summary;

/* Result of the latest stability/interface check. */
typedef struct {
    int64_t step;            /* step at which the check ran (0 = initial state) */
    double mass;             /* sum of rho over the grid (FP64) */
    double momx, momy;       /* sum of rho v (FP64) */
    double vmax;             /* max |v| */
    int64_t nan_count;       /* cells whose rho, vx or vy is NaN */
    double x_rear, x_front;  /* plug interfaces on the centreline; NaN unless exactly one liquid run */
    int32_t liquid_columns;  /* columns whose minimum density exceeds (rho_g + rho_l)/2 */
    int64_t rupture_step;    /* first check step with no liquid column; -1 before rupture */
    int64_t unstable_step;   /* first check step that failed; -1 if none */
} lbm_check_result;

/* Defaults: Carnahan-Starling a=1, b=4, R=1 at 0.85 Tc, k=1, kappa=0.001, paper MRT
   rates, rho_wall=rho_l, dp=0, extrapolated ends, walls, FP32 storage, check every
   1000 steps, v_limit 0.5, history of 4096 steps, automatic tiling. */
void lbm_params_default(lbm_params* p);

/* Validates the parameters, solves the EOS critical point and the Maxwell
   coexistence densities on the host (paper Sec. 2.2, verification paragraph) and
   returns a new context.  No device work.  tau > 1/2; 4 <= nx, ny; one copy
   of the distributions (9 * ny * nx rounded up to 64 columns, in the storage
   type) must stay below 4 GiB.  T_over_Tc >= 1 is allowed (single phase) but
   then lbm_init_plug is rejected. */
lbm_status lbm_create(int nx, int ny, double tau, const lbm_params* p, lbm_ctx** out);

/* Device bytes the caller must allocate and bind, and their alignment (256
   bytes; align may be NULL). */
lbm_status lbm_workspace(const lbm_ctx* ctx, size_t* bytes, size_t* align);

/* Binds caller-owned device memory (>= lbm_workspace bytes, 256-aligned) on
   the current HIP device and the hipStream_t (NULL = default stream) for all
   later launches.  Rebinding moves no data: initialise again afterwards.
   LBM_ENOMEM if bytes is too small; LBM_EINVAL if the pointer is null or not
   256-aligned, or if the first or last byte of the workspace is not device
   memory of the current device (host, pinned-host or unregistered memory,
   another device), checked on the host before anything is launched;
   LBM_EDEVICE when there is no current HIP device. */
lbm_status lbm_bind(lbm_ctx* ctx, void* device_ptr, size_t bytes, void* hip_stream);

/* Temperature, critical temperature, coexistence densities and wall density
   the context uses (host values, no device work). */
lbm_status lbm_state(const lbm_ctx* ctx, double* T, double* Tc, double* rho_g, double* rho_l,
                     double* rho_w);

/* Liquid plug of plug_len cells spanning the channel, centred at x_center
   (NaN: nx/4 + plug_len/2), and a liquid film of `film` rows on each wall
   (Sec. 2.3 and Sec. 3.1 of the paper), gas elsewhere, at the Maxwell densities,
   plus additive uniform noise of amplitude noise_amp: cell (x, y) adds
   noise_amp (2U - 1), U from the (y nx + x)-th output of SplitMix64(seed).
   A cell is liquid when x_center - plug_len/2 <= x < x_center + plug_len/2,
   or y < film, or y >= ny - film.  Distributions start at f_eq(rho, 0).
   Requires bind; 0 < plug_len <= nx, 0 <= 2 film < ny, T_over_Tc < 1. */
lbm_status lbm_init_plug(lbm_ctx* ctx, double plug_len, double film, double x_center,
                         double noise_amp, uint64_t seed);

/* Initial state from a host density field [ny][nx] (all > 0): f = f_eq(rho, 0). */
lbm_status lbm_init_density(lbm_ctx* ctx, const double* rho);

/* Advances n >= 0 steps, asynchronously on the bound stream.  A stability and
   interface check (lbm_check_result) runs at every step that is a multiple of
   check_every: the step there also writes the density and velocity fields, and
   the call waits for the check's results (one host synchronisation per check).
   Returns LBM_EUNSTABLE, and stops, at the first failed check, and also at the
   end of a call on a state an earlier check found unstable.  Between checks the
   steps are replayed from captured HIP graphs (graph_steps launches per graph,
   and one graph for the rest of the call; lbm_capture makes them beforehand).
   Every step's wall diagnostics are reduced into the per-step summaries and
   time integrals on the device before the call returns its stream work, so
   lbm_wall_stress and lbm_stress_history see every step; the call itself does
   not wait for the device.  The fields and the check of a step that was not a
   check step are formed when lbm_fields, lbm_fields_device, lbm_components,
   lbm_check_state or lbm_save ask for them (by running that step again with
   field output, which leaves the state unchanged). */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* Captures, without launching anything or changing the state, the HIP graphs
   that lbm_step(ctx, n) called now would replay, so that the call issues no
   capture of its own (a capture costs milliseconds).  LBM_ESTATE before bind
   and initialisation. */
lbm_status lbm_capture(lbm_ctx* ctx, int64_t n);

/* Number of steps taken since the last initialisation. */
lbm_status lbm_step_count(const lbm_ctx* ctx, int64_t* steps);

/* Density and velocity v = u + F/(2 rho) of the last step (after an
   initialisation: the initial density and zero velocity), copied to caller-owned
   host arrays [ny][nx] (FP64).  Any pointer may be NULL.  Waits for the
   stream. */
lbm_status lbm_fields(lbm_ctx* ctx, double* rho, double* vx, double* vy);

/* The fields of lbm_fields copied to caller-owned device arrays [ny][nx] on the
   bound stream (asynchronously; e.g. torch tensors): FP64 when fp64 != 0, else
   FP32 (rounded to nearest).  Any pointer may be NULL.  LBM_ESTATE before an
   initialisation; LBM_EINVAL, before anything is copied, if an output is not
   aligned to its element size or its first or last element is not device
   memory of the current device. */
lbm_status lbm_fields_device(lbm_ctx* ctx, void* rho, void* vx, void* vy, int fp64);

/* Wall shear stress and wall pressure of the last step along both walls
   (host arrays of nx doubles, any may be NULL) and that step's summary
   (may be NULL).  Before the first step they are zero. */
lbm_status lbm_wall_stress(lbm_ctx* ctx, double* tau_bot, double* tau_top, double* p_bot,
                           double* p_top, lbm_stress_summary* s);

/* The last min(cap, steps, history_cap) per-step summaries, oldest first. */
lbm_status lbm_stress_history(lbm_ctx* ctx, lbm_stress_summary* buf, int64_t cap, int64_t* n_out);

/* Stability/interface check of the current step: the one that already ran
   there, or else one run now (forming the step's fields first; one host
   synchronisation).  A check that finds NaN or |v| > v_limit sets
   unstable_step in the result and still returns LBM_OK.  Before bind and
   initialisation: the zero result. */
lbm_status lbm_check_state(lbm_ctx* ctx, lbm_check_result* out);

/* For callers that must not allocate memory (serving loops, harnesses that
   forbid allocation): lbm_check_state without any allocation.  Its first check
   allocates nothing: lbm_check_state stages its results in a pinned host
   buffer it allocates on first use, while this call keeps its device scratch
   (reduction partials, per-column minima and centreline densities, and the
   interface summary, which it forms on the device) in a static device array
   of the library and copies nine doubles back.  Same result as
   lbm_check_state, bit for bit.  The array holds the columns of lattices with
   nx <= 16384 (about 280 KB on each GPU the library runs on, kept until the
   process ends); LBM_EINVAL for wider lattices, before anything is launched.
   LBM_ESTATE before bind and initialisation.  Waits for the bound stream.
   All calls on one GPU share the array: calls that overlap in time on one GPU
   (from several threads, or on several streams) race and must not be made. */
lbm_status lbm_check_state_noalloc(lbm_ctx* ctx, lbm_check_result* out);

/* Tile autotuner of the tile schedule: times trial_steps launches of every
   tile shape (output rows x waves per block: 8x4, 12x4, 20x4, 28x4, 12x8,
   20x8, 28x8) on the current state and keeps the fastest for later steps.
   It also times two steps per launch (fused_steps = 2; not for F16R) and
   keeps them when they take less time per step, as on grids too small to fill
   the chip; otherwise it sets one step per launch.  Trials read the current
   state and write only scratch (the other distribution buffer and flushed
   wall-ring slots), so the state, fields and wall diagnostics are unchanged,
   and results do not depend on the choice (the kernels are bit-identical).
   Outputs (any may be NULL): the chosen one-step shape (also used for the
   single steps a two-step run needs) and the mean time per step in
   microseconds of the chosen configuration; lbm_launch_config reports
   whether two steps per launch were chosen.  Blocks until done.  LBM_EINVAL
   for other schedules or F64T. */
lbm_status lbm_autotune(lbm_ctx* ctx, int trial_steps, int* tile_rows, int* tile_waves, double* us_per_step);

/* The launch configuration in use: tile shape, steps per launch (1 or 2) and
   steps per captured graph (0: graphs off).  Any pointer may be NULL. */
lbm_status lbm_launch_config(const lbm_ctx* ctx, int* tile_rows, int* tile_waves, int* fused_steps,
                             int* graph_steps);

/* Reverse-mode sensitivities (adjoint) of the wall-shear objective
   J = sum over steps, walls and columns of tau_w^2 (the time integral of
   squared wall shear, int_tau2 of lbm_stress_summary; Figs. 3, 5 and 8 and
   Sec. 3.2-3.3 study the wall stresses against the pressure drop and the
   fluid), with respect to theta = (dp, a, b, T), T the absolute temperature.
   The initial state and the wall ghost density are held fixed, as for
   lbm_set_tangent.  One backward sweep gives all four derivatives: each
   adjoint step is the exact transpose of the step of eq. 2.1 with the force
   of eq. 2.17 (halfway bounce-back, extrapolated or periodic ends and wetting
   ghost rows included), run backwards from the last step.

   Memory: nsteps steps are recorded with one checkpoint of the state every
   `segment` steps (0 picks ceil(sqrt(nsteps))); the backward sweep recomputes
   each segment from its checkpoint, storing per step the forward fields the
   adjoint step reads (two segments' worth, so that one is recomputed while
   the other is swept).  The adjoint workspace holds ceil(nsteps/segment) + 2
   states, 2 x segment x (5 x ny x pitch + 4 x nx) values and two adjoint
   fields (9 x ny x pitch) of the arithmetic type, 2 x segment x 2 x nx FP64
   wall shears and small scratch; it is
   caller-owned device memory like the main workspace, 256-byte aligned, and
   bound once (the same pointer checks as lbm_bind).  Storage F64, F32 or
   F32D with the tile schedule; otherwise LBM_EINVAL. */
lbm_status lbm_adjoint_workspace(const lbm_ctx* ctx, int64_t nsteps, int64_t segment, size_t* bytes);
lbm_status lbm_adjoint_bind(lbm_ctx* ctx, void* device_ptr, size_t bytes, int64_t nsteps, int64_t segment);

/* The objective of the adjoint (after lbm_adjoint_bind, before
   lbm_adjoint_forward; changing it drops the record).  LBM_J_SUM_TAU2 (the
   default): J = sum over steps, walls and columns of tau_w^2 (int_tau2).
   LBM_J_PEAK_TAU2: J = sum over steps of the largest tau_w^2 over both walls
   and all columns (int_peak_tau2, the time-integrated squared peak wall
   shear); its gradient takes each step's derivative at the first (wall,
   column) holding the peak, which is the derivative wherever the peak is
   unique.  LBM_EINVAL for another value. */
typedef enum { LBM_J_SUM_TAU2 = 0, LBM_J_PEAK_TAU2 = 1 } lbm_adjoint_objective_kind;
lbm_status lbm_adjoint_objective(lbm_ctx* ctx, int objective);

/* Runs the next nsteps steps from the lattice's current state (through
   lbm_step, so checks and summaries proceed as usual) and records the
   checkpoints.  *J (may be NULL) receives J over these steps.  Errors of
   lbm_step (LBM_EUNSTABLE) are returned as they are; the record is then
   incomplete and lbm_adjoint_backward refuses it (LBM_ESTATE). */
lbm_status lbm_adjoint_forward(lbm_ctx* ctx, double* J);

/* Backward sweep over the recorded steps: grad[4] = seed * dJ/d(dp, a, b, T).
   For PR, dJ/da and dJ/db are NaN (alpha(T) depends on the critical
   temperature and with it on a and b).  Host grad; blocks until done.  The
   record stays valid, so the sweep can be repeated with another seed. */
lbm_status lbm_adjoint_backward(lbm_ctx* ctx, double seed, double* grad);

/* After lbm_adjoint_backward: seed * dJ/df*_i(x) of the recorded run's initial
   post-collision state, host FP64 [9][ny][nx]. */
lbm_status lbm_adjoint_state_gradient(lbm_ctx* ctx, double* dJ_df);

/* Restarts the running extremes of the wall summaries (run_tau_*, run_p_*)
   from the next step on, so that their spans cover a chosen window (for
   example the rupture, without the start-up transient).  Time integrals and
   step counts are unchanged.  Enqueued on the bound stream. */
lbm_status lbm_reset_stress_extremes(lbm_ctx* ctx);

/* One connected region of liquid cells (rho > threshold) of a density field.
   Sec. 3.2 and 3.3 of the paper follow the droplets that break away from the
   plug and the wall films during rupture ("aerosols") and their mass; here an
   aerosol is a component with no cell on a wall row. */
typedef struct {
    int64_t first_cell;  /* smallest row-major index y * nx + x among its cells (identifies it) */
    int32_t cells;       /* number of cells */
    int32_t wall;        /* 1 when a cell lies on row 0 or row ny - 1 and the walls are present */
    double mass;         /* sum of rho over its cells */
    double excess_mass;  /* sum of (rho - rho_g) over its cells */
    double cx, cy;       /* centroid; across a periodic direction each cell counts at its nearest
                            image to the first cell, and the mean is wrapped into [0, n) */
} lbm_component;

typedef struct {
    int64_t step;             /* step of the field (0 for lbm_components_field) */
    int64_t components;       /* liquid components */
    int64_t aerosols;         /* components with wall == 0 */
    int64_t aerosol_cells;
    double threshold;         /* the density threshold used */
    double liquid_mass;       /* sum of rho over all liquid cells */
    double aerosol_mass;      /* sum of mass over the aerosols */
    double aerosol_excess_mass;
} lbm_aerosol_summary;

/* Liquid components of the density of the last step (as lbm_fields returns
   it), labelled on the host after one copy of the field.  threshold NaN
   selects (rho_g + rho_l) / 2; connectivity is 4 (edge neighbours) or 8 (and
   corners); periodic ends (and periodic y) join opposite edges.  Writes the
   first min(cap, count) components in increasing first_cell to out (out may
   be NULL when cap is 0), the count to *n_out and the totals to *summary
   (either may be NULL).  LBM_EINVAL for a bad connectivity or a threshold
   that cannot be chosen (NaN above the critical temperature). */
lbm_status lbm_components(lbm_ctx* ctx, double threshold, int connectivity, lbm_component* out, int64_t cap,
                          int64_t* n_out, lbm_aerosol_summary* summary);

/* The same on a caller-owned host field rho[ny][nx] (no context, no device);
   y_periodic = 1 means there are no walls.  rho_g enters excess_mass only. */
lbm_status lbm_components_field(const double* rho, int nx, int ny, int x_periodic, int y_periodic, double threshold,
                                double rho_g, int connectivity, lbm_component* out, int64_t cap, int64_t* n_out,
                                lbm_aerosol_summary* summary);

/* F64T storage: the direction of the parameter tangent, dtheta = (d dp, d a,
   d b, d T) with T the absolute temperature (T_over_Tc times the critical
   temperature of the unperturbed a, b, R).  The initial state and the wall
   ghost density are held fixed, so the tangents start at zero at every
   initialisation and d int_tau2 is the derivative of the time integral of
   squared wall shear.  For PR, d a and d b must be 0 (its alpha depends on the
   critical temperature).  Takes effect from the next lbm_step; LBM_EINVAL for
   another storage type or non-finite entries. */
lbm_status lbm_set_tangent(lbm_ctx* ctx, const double* dtheta);
/* F64T storage: the tangents of the post-collision distributions [9][ny][nx]. */
lbm_status lbm_get_f_tangent(lbm_ctx* ctx, double* df);

/* Post-collision distributions as FP64 host arrays [9][ny][nx]
   (decoded from the storage type) / replaced from such an array (encoded with
   round-to-nearest-even).  lbm_set_f keeps the step count and history. */
lbm_status lbm_get_f(lbm_ctx* ctx, double* f);
lbm_status lbm_set_f(lbm_ctx* ctx, const double* f);

/* Frees a context (a no-op for a context owned by a batch). */
/* Checkpoint and resume (a run split over jobs, as the 100000-step runs of
   Sec. 3 may need).  lbm_save writes the current distributions, the step
   count, the latest check, the fields of the last step, the wall-stress time
   integrals and running extremes (after flushing the pending steps), the F16R
   step counter and the F64T tangent direction to `path`, with an FNV-1a hash
   of the content.  lbm_load reads such a file into a bound context created
   with the same nx, ny, tau and parameters (else LBM_EINVAL, also for a
   missing, short or corrupt file) and continues from there: stepping the
   loaded context gives bit for bit the states, checks and time integrals the
   saved run would have given.  Not kept: the per-step history and the wall
   arrays of the saved steps (the history restarts with the next step; the wall
   arrays read zero until then) and any adjoint record.  Batch cases are not
   saved or loaded on their own (LBM_ESTATE).  Both block until done. */
lbm_status lbm_save(lbm_ctx* ctx, const char* path);
lbm_status lbm_load(lbm_ctx* ctx, const char* path);

void lbm_destroy(lbm_ctx* ctx);
const char* lbm_last_error(const lbm_ctx* ctx);

/* ---- Batches -------------------------------------------------------------
   The studies of Sec. 3.3 (Figs 10-12) sweep the pressure drop, the plug and
   the film thickness over many cases.  A batch advances many independent
   lattices, of any sizes and parameters, with one kernel launch per step for
   all of them (the tile schedule over the concatenated tiles), so small cases
   share the fixed cost of a launch.  Every case is an ordinary context (init,
   fields, wall stress, history, checks, components, get_f/set_f all work on
   it) except that only lbm_batch_step advances it. */
typedef struct lbm_batch lbm_batch;

/* n cases of sizes nx[k] x ny[k], relaxation times tau[k] and parameters
   params[k] (all host arrays of n entries).  storage, eos, tile_rows,
   tile_waves and check_every must be equal across the cases and schedule must
   be 0; otherwise LBM_EINVAL, as for any case lbm_create would reject. */
lbm_status lbm_batch_create(int n, const int* nx, const int* ny, const double* tau, const lbm_params* params,
                            lbm_batch** out);
/* Device bytes the batch needs (all cases' workspaces and the per-case launch table). */
lbm_status lbm_batch_workspace(const lbm_batch* b, size_t* bytes);
/* Binds caller-owned device memory (256-byte aligned, at least lbm_batch_workspace
   bytes; the caller keeps ownership) and a stream to the batch and all its
   cases, and uploads the launch table (synchronises the stream).  The same
   pointer checks as lbm_bind. */
lbm_status lbm_batch_bind(lbm_batch* b, void* device_ptr, size_t bytes, void* hip_stream);
/* Borrowed handle of case k (0 <= k < n), valid until lbm_batch_destroy. */
lbm_status lbm_batch_case(lbm_batch* b, int k, lbm_ctx** ctx);
/* Advances every case by n >= 0 steps, one launch per step (two steps per
   launch when the cases were created with fused_steps = 2 or the autotuner
   chose it; checks and the last step of a call are one-step launches), with each case's
   checks at the common check cadence, asynchronously as lbm_step (graphs
   between checks, wall summaries reduced on the device, one wait per check;
   a case's fields and check at another step are formed when asked for).  All
   cases must be initialised and have equal step counts (initialise them
   together).  On a failed check returns that status, stops, and sets
   *failed_case (may be NULL) to the case index (-1 otherwise); a call on a
   batch with a case found unstable before returns LBM_EUNSTABLE too. */
lbm_status lbm_batch_step(lbm_batch* b, int64_t n, int* failed_case);
/* As lbm_capture, for lbm_batch_step(b, n). */
lbm_status lbm_batch_capture(lbm_batch* b, int64_t n);
/* The tile autotuner for a batch: one trial launch covers every case's tiles
   for a shape (the cases share one kernel), then two steps per launch are timed
   as well (storage types with the two-step kernel), and the fastest is kept for
   all cases (lbm_launch_config of a case reports it).  As lbm_autotune
   otherwise; every case must be initialised. */
lbm_status lbm_batch_autotune(lbm_batch* b, int trial_steps, int* tile_rows, int* tile_waves, double* us_per_step);

void lbm_batch_destroy(lbm_batch* b);
const char* lbm_batch_last_error(const lbm_batch* b);

#ifdef __cplusplus
}
#endif
#endif
