// lbm_internal.hpp -- declarations shared by the library's host code and its
// HIP kernels.  Not part of the public C ABI (include/lbm.h).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>

#include "lbm.h"

namespace lbm {

// Output columns per 64-lane wavefront strip: each wave covers 64 consecutive
// columns, of which the outer two on each side are the radius-2 halo that the
// force stencil grad(lap rho) needs.
constexpr int kStripOut = 60;
constexpr int kWavesPerBlock = 4;
// One step's slot of the wall ring: per wall column, FP64 wall shear [2][nx],
// wall pressure [2][nx] and the wall shear's tangent [2][nx] (zero unless the
// storage is tangent-linear).
constexpr int kWallSlotVals = 6;
constexpr int kScheduleTile = 0;   // block-per-tile kernel with LDS-coupled phases
constexpr int kScheduleMarch = 1;  // wave-per-strip row march with a register window
constexpr int kSchedulePipe = 2;   // persistent blocks taking tiles by ticket, next tile's loads in flight
constexpr int kTicketGroups = 8;   // one ticket counter per XCD
constexpr int kTicketStride = 32;  // counters 256 bytes apart (in 64-bit words)

// The step coefficients rounded to FP32 on the host, so FP32 kernels read them
// as scalars instead of converting the FP64 values in every wave.
struct CoefF32 {
    float tau, s_e, s_eps, s_q, s_j, s_v, k2, kappa, g, nu, RT, a_eff, b, rho_w, rho0;
};

// Tangents of the step coefficients along the parameter direction of the
// tangent-linear storage (zero otherwise).  Only g, RT, a_eff and b move.
struct CoefTangent {
    double tau, s_e, s_eps, s_q, s_j, s_v, k2, kappa, g, nu, RT, a_eff, b, rho_w, rho0;
};

// Everything one launch of the step kernel needs, passed by value.
struct StepArgs {
    const void* fin;          // post-collision distributions of the previous step
    void* fout;               // new post-collision distributions
    int nx, ny, pitch;        // pitch: elements per row of a distribution plane
    long long plane;          // elements per plane (pitch * ny)
    int nstrip, nchunk, ty;   // x strips, y chunks, output rows per chunk/tile
    int schedule;             // kScheduleTile or kScheduleMarch
    int tile_waves;           // waves per tile block (4 or 8)
    int xper, yper;
    double tau, s_e, s_eps, s_q, s_j, s_v;
    double k2, kappa, g, nu;
    double RT, a_eff, b;      // EOS: R T, a * alpha(T), b
    double rho_w;             // wall ghost density
    double rho0;              // shifted storage (F32S/F16S/F16R/BF16S): the shift unit q, rho0 / 9 on a 2^-24 grid
    CoefF32 cf;               // the coefficients above, rounded to FP32
    CoefTangent ct;           // their tangents (tangent-linear storage)
    double* tau_w;            // [2][nx] wall shear of this step (its slot of the wall ring)
    double* p_w;              // [2][nx] wall pressure of this step
    double* dtau_w;           // [2][nx] tangent of the wall shear of this step
    double* ring;             // batch launches: base of the case's wall ring (slots of kWallSlotVals * nx)
    unsigned long long* tickets;  // kTicketGroups counters, kTicketStride apart (pipelined schedule)
    long long launch;         // launches since the counters were zeroed (pipelined schedule)
    int pipe_blocks;          // grid of the pipelined schedule
    double* rho_out;          // emitted fields [ny][nx] (only read when emitting)
    double* vx_out;
    double* vy_out;
    void* save;               // the adjoint's fields of this step (launch_step_save only)
    uint32_t* sr;             // F16R: two step counters; a launch reads sr[sr_par] and writes sr[1 - sr_par]
    int sr_par;               // (batch launches take the parity from their own argument)
};

hipError_t launch_step(const StepArgs& a, int storage, int eos, bool emit, hipStream_t s);
// Per storage type (one translation unit each, lbm_step_<type>.hip): the step,
// batch-step and pipelined-grid launchers that launch_step, launch_step_batch
// and pipe_grid dispatch to.
#define LBM_DECLARE_STORAGE_LAUNCHERS(NAME)                                                                   \
    hipError_t launch_step_##NAME(const StepArgs& a, int eos, bool emit, hipStream_t s);                     \
    hipError_t launch_batch_##NAME(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, \
                                   int parity, int slot, int eos, int ty, int waves, bool emit, hipStream_t s); \
    hipError_t pipe_grid_##NAME(int eos, int ty, int waves, int* blocks);                                     \
    hipError_t launch_step2_##NAME(const StepArgs& a, int eos, bool emit, hipStream_t s);                    \
    hipError_t launch_batch2_##NAME(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, \
                                    int parity, int slot, int eos, bool emit, hipStream_t s);
LBM_DECLARE_STORAGE_LAUNCHERS(f64)
LBM_DECLARE_STORAGE_LAUNCHERS(f32)
LBM_DECLARE_STORAGE_LAUNCHERS(f16s)
LBM_DECLARE_STORAGE_LAUNCHERS(bf16s)
LBM_DECLARE_STORAGE_LAUNCHERS(f32d)
LBM_DECLARE_STORAGE_LAUNCHERS(f32s)
#undef LBM_DECLARE_STORAGE_LAUNCHERS
hipError_t launch_step_f64t(const StepArgs& a, int eos, bool emit, hipStream_t s);
// FP16 storage with stochastic rounding (lbm_step_f16r.hip): the tile schedule
// and batches only.
hipError_t launch_step_f16r(const StepArgs& a, int eos, bool emit, hipStream_t s);
hipError_t launch_batch_f16r(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, int parity,
                             int slot, int eos, int ty, int waves, bool emit, hipStream_t s);
// Two steps in one launch (temporal blocking, the tile schedule's two-step kernel):
// reads a.fin, writes a.fout after two steps; the wall arrays of the first step
// go to a.tau_w/p_w/dtau_w and those of the second kWallSlotVals * nx further on.
// Not for F64T storage.
hipError_t launch_step2(const StepArgs& a, int storage, int eos, bool emit, hipStream_t s);
// Tiles of the two-step kernel: 54 output columns (a 5-column halo each side) by
// kTile2Rows rows (kTile2RowsF64 with FP64 arithmetic).
constexpr int kStrip2Out = 54;
constexpr int kTile2Rows = 14, kTile2RowsF64 = 6;
inline int tiles2(int nx, int ny, int rows) { return ((nx + kStrip2Out - 1) / kStrip2Out) * ((ny + rows - 1) / rows); }
// Two steps of many lattices in one launch (as launch_step_batch, with the
// two-step tiles: tile_start counts tiles2 per case); the two steps' wall arrays
// go to ring slots slot and slot + 1.  Not for F64T or F16R storage.
hipError_t launch_step2_batch(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, int parity,
                              int slot, int storage, int eos, bool emit, hipStream_t s);
// One step of many lattices in one launch (tile schedule): cases[c] holds case
// c's arguments with both distribution buffers (f[0] as fin, f[1] as fout) and
// the base of its wall ring; tile_start[c] is its first tile (device arrays).
hipError_t launch_step_batch(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, int parity,
                             int slot, int storage, int eos, int ty, int waves, bool emit, hipStream_t s);
// Resident blocks of the pipelined kernel for this configuration: CUs times the
// blocks one CU holds at once.
hipError_t pipe_grid(int storage, int eos, int ty, int waves, int* blocks);
hipError_t launch_init(const double* rho, void* f, int nx, int ny, int pitch, long long plane,
                       int storage, double q, hipStream_t s);
hipError_t launch_fill(double* p, double v, long long n, hipStream_t s);
// out[i] = (float)in[i], i < n.
hipError_t launch_to_f32(const double* in, float* out, long long n, hipStream_t s);
// Stage 1+2 FP64 reduction over the emitted fields into out[5]:
// sum rho, sum rho vx, sum rho vy, max |v|^2, NaN count.
hipError_t launch_field_reduce(const double* rho, const double* vx, const double* vy, long long n,
                               double* partials, int nblocks, double* out, hipStream_t s);
// Per column: minimum density over y and the centreline density.
hipError_t launch_column_scan(const double* rho, int nx, int ny, double* colmin, double* centre,
                              hipStream_t s);
// Reduces the first `nsteps` slots of the wall ring into the history ring, then
// accumulates the running time integrals and running extremes acc[kWallAccVals] in
// step order.  A block per (wall, step) reduces that wall's columns (extremes with
// their smallest column, sums of squares) into scratch[step][wall][kWallPartVals];
// the last block to finish (a ticket counter in the accumulator block, zero between
// flushes) integrates over the steps.  The history takes its step numbers from the
// accumulator block (acc[kAccNextStep], the first step not yet flushed), which the
// flush advances, so a flush launch does not depend on the step count and can be
// captured in a graph.
constexpr int kAccTicket = 16;    // acc index holding the flush's ticket (an unsigned)
constexpr int kAccNextStep = 17;  // acc index holding the next step to flush (an integer in a double)
hipError_t launch_wall_reduce(const double* ring, int nsteps, int nx, lbm_stress_summary* hist, int hist_cap,
                              double* scratch, double* acc, hipStream_t s);
// The wall ring, history, scratch and accumulators of one lattice.
struct WallFlush {
    const double* ring;
    int nx;
    lbm_stress_summary* hist;
    int hist_cap;
    double* scratch;
    double* acc;
};
// launch_wall_reduce for the ncases lattices of tbl (device array) at once;
// they have stepped together, so nsteps and first_step are shared.
hipError_t launch_wall_reduce_batch(const WallFlush* tbl, int ncases, int nsteps, hipStream_t s);

// Reverse-mode (adjoint) step (lbm_adjoint.hip).  Tiles of 64 columns give 60
// outputs (a 2-column halo on each side) and ty output rows.
constexpr int kAdjStripOut = 60;
// Forward quantities of one step that its adjoint reads, written by the step
// itself during the backward sweep's recompute (arithmetic type, planes of
// `plane` elements at the distributions' row pitch): rho, u = (j + tau F)/rho
// (two planes), grad lap rho (two planes); then the velocity shift
// v_x = (j_x + F_x/2)/rho of the wall rows 0, 1, ny - 2, ny - 1 as 4 x nx.
constexpr int kAdjFieldPlanes = 5;
inline long long adjoint_field_elems(long long plane, int nx) { return kAdjFieldPlanes * plane + 4LL * nx; }
// One step of the tile schedule (fixed 8-row, 4-wave tiles) that also writes
// the adjoint's fields of the step to a.save.  F64, F32 and F32D storage.
hipError_t launch_step_save(const StepArgs& a, int storage, int eos, hipStream_t s);
struct AdjArgs {
    StepArgs s;            // the step's coefficients and geometry
    const void* fld;       // the step's forward fields (layout above)
    const void* lam_in;    // dJ/df of the next step's pulled populations [9][ny][pitch] (arithmetic type)
    void* lam_out;         // the same for this step
    const double* tau_w;   // [2][nx] this step's wall shear (from its forward recompute)
    const double* seed;    // [2][nx] dJ/dtau_w of this step, or null for J = sum tau_w^2 (seed 2 tau_w)
    double* partial;       // [blocks][4]: sum F~_x, sum phi~ dphi/dRT, dphi/da_eff, dphi/db
    int nstrip;            // 60-column strips
    int ty;                // output rows per tile (adjoint_tile_shape)
    int waves;             // waves per tile block
};
hipError_t launch_adjoint(const AdjArgs& A, int storage, int eos, hipStream_t s);
// Seeds of the peak objective J = sum over steps of max over walls and columns of
// tau_w^2, for `steps` consecutive steps of [2][nx] wall shears: seed = 2 tau_w at
// the first (wall, column) where tau_w^2 is largest, 0 elsewhere.
hipError_t launch_peak_seed(const double* tau_w, double* seed, int nx, int steps, hipStream_t s);
// acc[0..3] += the parameter sums of `launches` consecutive adjoint launches
// (partial: [launches][blocks][4]), launch totals added in launch order; red is
// scratch of launches x 4 doubles.
hipError_t launch_adjoint_reduce(const double* partial, int launches, int blocks, double* red, double* acc,
                                 hipStream_t s);
// dJ/df* of a state from the adjoint of the step that read it, as FP64 [9][ny][nx].
hipError_t launch_adjoint_gather(const void* lam, const StepArgs& a, int storage, double* out, hipStream_t s);
int adjoint_blocks(int nx, int ny, int ty);

constexpr int kFieldReduceBlocks = 512;

// The check of lbm_check_state_noalloc (lbm_noalloc.hip), whose device scratch is a
// static array of the library holding the reduction partials and the column scans
// of up to kNoAllocMaxNx columns.  noalloc_setup resolves the array's address on the
// current device (once per device); noalloc_check reduces the fields rho, vx, vy
// [ny][nx] of `device` on stream s and returns, after waiting for s: [0..4] sum rho,
// sum rho vx, sum rho vy, max |v|^2, NaN count; [5] liquid columns; [6] x_rear;
// [7] x_front; [8] centreline liquid runs.  Calls that overlap on one device race.
constexpr int kNoAllocMaxNx = 16384;
hipError_t noalloc_setup();
hipError_t noalloc_check(int device, const double* rho, const double* vx, const double* vy, int nx, int ny,
                         double mid, double* host9, hipStream_t s);
constexpr int kWallPartVals = 10;  // per step and wall: tau max, its x, tau min, its x, p max, its x, p min, its x,
                                   // sum tau^2, sum 2 tau dtau (the flush's scratch holds [steps][2][kWallPartVals])
constexpr int kWallAccVals = 11;      // int peak tau^2, int sum tau^2, running tau/p max/min per wall, d int tau^2
static_assert(kWallAccVals <= kAccTicket && kAccNextStep < 32, "the accumulator block holds 32 doubles");

// Liquid components of a host density field (lbm_post.cpp).
lbm_status label_components(const double* rho, int nx, int ny, bool xper, bool yper, double threshold, double rho_g,
                            int connectivity, lbm_component* out, int64_t cap, int64_t* n_out,
                            lbm_aerosol_summary* summary);

}  // namespace lbm
