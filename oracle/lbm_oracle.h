/*
 * lbm_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference of the EOS-based multiphase MRT lattice
 * Boltzmann time step of He, Qin, Chen & Wen, "Numerical simulation of
 * pulmonary airway reopening by the EOS-based multiphase lattice Boltzmann
 * method" (arXiv 2103.08301), Sec. 2.  It exists so that tests can check the
 * GPU library against an independent, obviously-correct implementation.
 *
 * Only tests/, the package's smoke() entry and the bench's CPU-baseline leg
 * may load this library.  It shares no code, header, table or helper with the
 * GPU library; neither includes, links or imports the other.
 *
 * Every floating-point result is FP64, compiled without FMA contraction.
 * Grids are row-major with x fastest: field[y][x]; distributions are
 * f[i][y][x] (structure of arrays), i = 0..8 in the D2Q9 order
 *   e0=(0,0) e1=(1,0) e2=(0,1) e3=(-1,0) e4=(0,-1)
 *   e5=(1,1) e6=(-1,1) e7=(-1,-1) e8=(1,-1).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_EOS_CS = 0, ORC_EOS_PR = 1 };

/* Status codes (0 = ok). */
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EUNSTABLE = -4 };

typedef struct {
    int eos;            /* ORC_EOS_CS (Carnahan-Starling) or ORC_EOS_PR (Peng-Robinson, eq. 2.18) */
    double a, b, R;     /* EOS constants */
    double omega;       /* PR acentric factor (Sec. 2.2 verification paragraph) */
    double T_over_Tc;   /* temperature as a fraction of the EOS's critical temperature */
    double k;           /* proportional coefficient, eqs. 2.13-2.17 */
    double kappa;       /* gradient coefficient, eqs. 2.3 and 2.17 */
    double tau;         /* relaxation time; s_v = 1/tau (Sec. 2.1) */
    double s_e, s_eps, s_q;  /* MRT rates (Sec. 2.1) */
    double s_j;         /* rate on the momentum rows; <= 0 selects 1/tau */
    double rho_wall;    /* virtual density in the wall ghost rows; NaN selects rho_l */
    double dp;          /* pressure drop along x; body force density dp/nx */
    int x_periodic;     /* 1: periodic in x; 0: extrapolated (zero-gradient) ends */
    int y_periodic;     /* 1: periodic in y (no walls); 0: halfway bounce-back walls */
    int check_every;    /* stability check cadence in steps (>= 1) */
    double v_limit;     /* |v| above this (or a NaN) at a check is an instability */
    int forcing;        /* ORC_FORCING_VELOCITY_SHIFT (Sec. 2.2, the method) or, for comparison
                           only, ORC_FORCING_EXACT_DIFFERENCE */
} orc_params;

/* How the force enters the collision.  The method of the paper shifts the
   equilibrium velocity (Sec. 2.2).  The exact difference method of Kupershtokh,
   Medvedev & Karpov (Comput. Math. Appl. 58, 2009) relaxes towards the
   equilibrium at u = j/rho and then adds f_eq(rho, u + F/rho) - f_eq(rho, u),
   which leaves the steady state independent of tau; it is here only to compare
   the two, and the GPU library implements the velocity shift alone. */
enum { ORC_FORCING_VELOCITY_SHIFT = 0, ORC_FORCING_EXACT_DIFFERENCE = 1 };

typedef struct {
    int64_t step;                       /* 1-based index of the step these values belong to */
    double tau_max[2], tau_min[2];      /* [0] bottom wall, [1] top wall */
    double p_max[2], p_min[2];
    int32_t x_tau_max[2], x_tau_min[2]; /* smallest x attaining the extreme */
    int32_t x_p_max[2], x_p_min[2];
    double sum_tau2;                    /* sum over both walls and all x of tau_w^2 */
    double int_peak_tau2;               /* running sum over steps of max_{wall,x} tau_w^2 */
    double int_tau2;                    /* running sum over steps of sum_tau2 */
    double run_tau_max[2], run_tau_min[2];  /* extremes over x and over steps 1..step (the
                                               max - min spans of Sec. 3.2-3.3) */
    double run_p_max[2], run_p_min[2];
} orc_summary;

typedef struct orc_sim orc_sim;

/* One 4- or 8-connected component of the cells with rho > threshold
   (a liquid region; Sec. 3.2-3.3 call a detached one an aerosol droplet). */
typedef struct {
    int64_t first_cell;   /* smallest row-major index y * nx + x among its cells */
    int32_t cells;        /* number of cells */
    int32_t wall;         /* 1 if a cell lies on row 0 or row ny-1 and walls are present */
    double mass;          /* sum of rho over its cells */
    double excess_mass;   /* sum of (rho - rho_g) over its cells */
    double cx, cy;        /* centroid; across a periodic direction each cell is taken at its
                             nearest image to the first cell, and the mean wrapped into [0, n) */
} orc_component;

void   orc_params_default(orc_params* p);

/* Equation of state (Sec. 2.2; eq. 2.18 for PR). */
int    orc_critical(const orc_params* p, double* rho_c, double* T_c);
double orc_alpha(const orc_params* p, double T, double T_c);
double orc_p0(const orc_params* p, double T, double rho);
double orc_dp0(const orc_params* p, double T, double rho, int order);   /* order 1 or 2 */
int    orc_coexistence(const orc_params* p, double T, double* rho_g, double* rho_l, double* p_star);

/* Single-node and stencil building blocks, exposed for tests. */
void   orc_velocities(int i, int* ex, int* ey, double* w);
void   orc_moment_matrix(double* M81);                    /* row-major 9x9 */
void   orc_equilibrium(double rho, double ux, double uy, double* feq9);
void   orc_collide_node(const orc_params* p, const double* f9, double Fx, double Fy,
                        double* fout9, double* rho, double* vx, double* vy);
void   orc_grad_field(const double* a, int w, int h, double* gx, double* gy);
void   orc_lap_field(const double* a, int w, int h, double* lap);
uint64_t orc_splitmix64(uint64_t seed, uint64_t counter);   /* counter-th output (0-based) */
int    orc_threads(void);                                  /* OpenMP threads a step uses */

/* Time stepper. */
int    orc_create(int nx, int ny, const orc_params* p, orc_sim** out);
void   orc_destroy(orc_sim* s);
int    orc_state(const orc_sim* s, double* T, double* Tc, double* rho_g, double* rho_l, double* rho_w);
int    orc_init_plug(orc_sim* s, double plug_len, double film, double x_center,
                     double noise_amp, uint64_t seed);
int    orc_init_density(orc_sim* s, const double* rho);    /* f* = f^eq(rho, 0) */
void   orc_set_f(orc_sim* s, const double* f);             /* [9][ny][nx], post-collision */
void   orc_get_f(const orc_sim* s, double* f);
int    orc_step(orc_sim* s, int64_t n);
int64_t orc_step_count(const orc_sim* s);
int64_t orc_unstable_step(const orc_sim* s);
void   orc_fields(const orc_sim* s, double* rho, double* vx, double* vy);
void   orc_force(const orc_sim* s, double* Fx, double* Fy);
void   orc_wall(const orc_sim* s, double* tau_bot, double* tau_top, double* p_bot, double* p_top);
/* The force of eq. 2.17 (plus the body force dp/nx) and the wall pressure of
   the first fluid rows (isotropic part of eq. 2.8) of a given density field
   rho[ny][nx], evaluated by the stages a step runs after streaming: ghost ring
   and EOS field, Laplacian, force, wall pressure.  Fx, Fy: [ny][nx]; p_bot,
   p_top: [nx], left untouched with periodic y; any may be NULL.  It replaces
   the simulation's density and force fields (not its distributions): meant for
   a simulation used for nothing else. */
void   orc_eval_force(orc_sim* s, const double* rho, double* Fx, double* Fy, double* p_bot, double* p_top);
int64_t orc_history(const orc_sim* s, orc_summary* buf, int64_t cap);
void   orc_totals(const orc_sim* s, double* mass, double* momx, double* momy);
int    orc_interface(const orc_sim* s, double* x_rear, double* x_front, int* liquid_columns);

/* Components of an arbitrary field rho[ny][nx].  connectivity is 4 or 8;
   x_periodic / y_periodic join the opposite edges (y_periodic also means there
   are no walls).  Writes at most cap components, in increasing first_cell, and
   returns how many there are (or a negative status). */
int64_t orc_components_field(const double* rho, int nx, int ny, int x_periodic, int y_periodic, double threshold,
                             double rho_g, int connectivity, orc_component* out, int64_t cap);
/* The same on the simulation's density, threshold NaN = (rho_g + rho_l) / 2. */
int64_t orc_components(const orc_sim* s, double threshold, int connectivity, orc_component* out, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif
