// lbm_kernels.hip -- the library's small kernels (initialisation, fills, FP64
// field reductions, column scans, wall-summary reductions) and the dispatch of
// a step launch to the translation unit of its storage type.
#include "lbm_device.hpp"

namespace lbm {
namespace {

template <class CD>
__global__ void init_kernel(const double* __restrict__ rho, void* fv, int nx, int ny, int pitch, long long plane,
                            double q) {  // q: the shifted codecs' shift unit
    using S = typename CD::S;
    using C = typename CD::C;
    S* f = static_cast<S*>(fv);
    const long long n = (long long)nx * ny;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        const int y = int(c / nx), x = int(c - (long long)y * nx);
        const C r = C(rho[c]);
        S* p = f + (long long)y * pitch + x;
        CD::template store<0>(p + 0 * plane, CD::template work<0>(wgt<C>(0) * r, C(q)), C(q));
        CD::template store<1>(p + 1 * plane, CD::template work<1>(wgt<C>(1) * r, C(q)), C(q));
        CD::template store<2>(p + 2 * plane, CD::template work<2>(wgt<C>(2) * r, C(q)), C(q));
        CD::template store<3>(p + 3 * plane, CD::template work<3>(wgt<C>(3) * r, C(q)), C(q));
        CD::template store<4>(p + 4 * plane, CD::template work<4>(wgt<C>(4) * r, C(q)), C(q));
        CD::template store<5>(p + 5 * plane, CD::template work<5>(wgt<C>(5) * r, C(q)), C(q));
        CD::template store<6>(p + 6 * plane, CD::template work<6>(wgt<C>(6) * r, C(q)), C(q));
        CD::template store<7>(p + 7 * plane, CD::template work<7>(wgt<C>(7) * r, C(q)), C(q));
        CD::template store<8>(p + 8 * plane, CD::template work<8>(wgt<C>(8) * r, C(q)), C(q));
    }
}

__global__ void fill_kernel(double* p, double v, long long n) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x)
        p[c] = v;
}

__global__ void to_f32_kernel(const double* __restrict__ in, float* __restrict__ out, long long n) {
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x)
        out[c] = float(in[c]);
}

// Deterministic two-stage FP64 reduction.  Stage 1: block b reduces the
// contiguous range [b n/B, (b+1) n/B) with a fixed thread/LDS tree.
constexpr int kRedThreads = 256;

__device__ inline void block_reduce5(double (&v)[5], double (*sh)[kRedThreads]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 5; ++k) sh[k][t] = v[k];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
            sh[0][t] += sh[0][t + s];
            sh[1][t] += sh[1][t + s];
            sh[2][t] += sh[2][t + s];
            sh[3][t] = fmax(sh[3][t], sh[3][t + s]);
            sh[4][t] += sh[4][t + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] = sh[k][0];
}

__global__ __launch_bounds__(kRedThreads) void field_reduce_stage1(const double* __restrict__ rho,
                                                                   const double* __restrict__ vx,
                                                                   const double* __restrict__ vy, long long n,
                                                                   double* __restrict__ partials) {
    __shared__ double sh[5][kRedThreads];
    const long long lo = n * blockIdx.x / gridDim.x, hi = n * (blockIdx.x + 1) / gridDim.x;
    double v[5] = {0, 0, 0, 0, 0};
    for (long long c = lo + threadIdx.x; c < hi; c += kRedThreads) {
        const double r = rho[c], ux = vx[c], uy = vy[c];
        v[0] += r;
        v[1] += r * ux;
        v[2] += r * uy;
        const double u2 = ux * ux + uy * uy;
        if (u2 > v[3]) v[3] = u2;
        if (r != r || ux != ux || uy != uy) v[4] += 1.0;
    }
    block_reduce5(v, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) partials[blockIdx.x * 5 + k] = v[k];
}

__global__ __launch_bounds__(kRedThreads) void field_reduce_stage2(const double* __restrict__ partials, int nb,
                                                                   double* __restrict__ out) {
    __shared__ double sh[5][kRedThreads];
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads) {
        v[0] += partials[b * 5 + 0];
        v[1] += partials[b * 5 + 1];
        v[2] += partials[b * 5 + 2];
        v[3] = fmax(v[3], partials[b * 5 + 3]);
        v[4] += partials[b * 5 + 4];
    }
    block_reduce5(v, sh);
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k) out[k] = v[k];
}

// Per column: the minimum density over y and the centreline density.  A block
// takes 64 columns; its kColScanWaves waves take every kColScanWaves-th row
// (four loads in flight per lane), and wave 0 combines the partial minima (fmin
// is exact and order-free: it skips NaNs, and gives NaN only if every value is).
constexpr int kColScanWaves = 8;
__global__ __launch_bounds__(64 * kColScanWaves) void column_scan_kernel(const double* __restrict__ rho, int nx, int ny,
                                                                         double* __restrict__ colmin,
                                                                         double* __restrict__ centre) {
    __shared__ double sh[kColScanWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = blockIdx.x * 64 + lane;
    const int xc = x < nx ? x : nx - 1;  // lanes past the last column read a valid column and store nothing
    const double none = __builtin_nan("");  // fmin's identity: an all-NaN column stays NaN
    double m[4] = {none, none, none, none};
    int y = wave;
    for (; y + 3 * kColScanWaves < ny; y += 4 * kColScanWaves)
#pragma unroll
        for (int u = 0; u < 4; ++u) m[u] = fmin(m[u], rho[(long long)(y + u * kColScanWaves) * nx + xc]);
    for (; y < ny; y += kColScanWaves) m[0] = fmin(m[0], rho[(long long)y * nx + xc]);
    sh[wave][lane] = fmin(fmin(m[0], m[1]), fmin(m[2], m[3]));
    __syncthreads();
    if (wave != 0 || x >= nx) return;
    double r = sh[0][lane];
    for (int w = 1; w < kColScanWaves; ++w) r = fmin(r, sh[w][lane]);
    colmin[x] = r;
    if (ny % 2 == 0)
        centre[x] = 0.5 * (rho[(long long)(ny / 2 - 1) * nx + x] + rho[(long long)(ny / 2) * nx + x]);
    else
        centre[x] = rho[(long long)(ny / 2) * nx + x];
}

// Extremes with their columns: a strictly better value wins, an equal one keeps the
// smaller column, so any fixed combination order yields the smallest column on ties.
__device__ inline void comb_max(double& v, double& x, double ov, double ox) {
    if (ov > v || (ov == v && ox < x)) { v = ov; x = ox; }
}
__device__ inline void comb_min(double& v, double& x, double ov, double ox) {
    if (ov < v || (ov == v && ox < x)) { v = ov; x = ox; }
}

constexpr int kWallThreads = 256;  // threads of a flush block; the integration takes one per step (4 waves)
constexpr int kWallWaves = kWallThreads / 64;

// One wall of one step of the wall ring: extremes of tau_w and p_w with their columns
// (the smallest column on ties) and the sums of tau_w^2 and of its tangent, reduced
// lane-strided (sixteen columns' loads in flight per thread), then by wave butterflies,
// then over the waves in order.  Thread 0 writes the ten values to scratch[t][w].
// Every thread returns.
__device__ void wall_step_reduce(const WallFlush& f, int t, int w) {
    __shared__ double sh[kWallWaves][kWallPartVals];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nx = f.nx;
    const double* slot = f.ring + (long long)t * kWallSlotVals * nx;  // tau [2][nx], p [2][nx], dtau [2][nx]
    const double* tau = slot + (long long)w * nx;
    const double* pw = slot + (long long)(2 + w) * nx;
    const double* dtau = slot + (long long)(4 + w) * nx;
    double tmax = -INFINITY, xtmax = 1e300, tmin = INFINITY, xtmin = 1e300;
    double pmax = -INFINITY, xpmax = 1e300, pmin = INFINITY, xpmin = 1e300, ws = 0.0, wds = 0.0;
#pragma unroll 16
    for (int x = threadIdx.x; x < nx; x += kWallThreads) {
        const double tv = tau[x], pv = pw[x];
        comb_max(tmax, xtmax, tv, double(x));
        comb_min(tmin, xtmin, tv, double(x));
        comb_max(pmax, xpmax, pv, double(x));
        comb_min(pmin, xpmin, pv, double(x));
        ws += tv * tv;
        wds += 2.0 * tv * dtau[x];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        comb_max(tmax, xtmax, __shfl_xor(tmax, off, 64), __shfl_xor(xtmax, off, 64));
        comb_min(tmin, xtmin, __shfl_xor(tmin, off, 64), __shfl_xor(xtmin, off, 64));
        comb_max(pmax, xpmax, __shfl_xor(pmax, off, 64), __shfl_xor(xpmax, off, 64));
        comb_min(pmin, xpmin, __shfl_xor(pmin, off, 64), __shfl_xor(xpmin, off, 64));
        ws += __shfl_xor(ws, off, 64);
        wds += __shfl_xor(wds, off, 64);
    }
    if (lane == 0) {
        double* o = sh[wave];
        o[0] = tmax; o[1] = xtmax; o[2] = tmin; o[3] = xtmin;
        o[4] = pmax; o[5] = xpmax; o[6] = pmin; o[7] = xpmin; o[8] = ws; o[9] = wds;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[kWallPartVals];
        for (int q = 0; q < kWallPartVals; ++q) r[q] = sh[0][q];
        for (int v = 1; v < kWallWaves; ++v) {
            const double* o = sh[v];
            comb_max(r[0], r[1], o[0], o[1]);
            comb_min(r[2], r[3], o[2], o[3]);
            comb_max(r[4], r[5], o[4], o[5]);
            comb_min(r[6], r[7], o[6], o[7]);
            r[8] += o[8];
            r[9] += o[9];
        }
        double* o = f.scratch + ((long long)t * 2 + w) * kWallPartVals;
        for (int q = 0; q < kWallPartVals; ++q) o[q] = r[q];
    }
}

// The per-step summaries and the running time integrals and extremes of nsteps <=
// kWallThreads steps (thread per step).  A step's summary combines its two walls'
// partials (peak of tau_w^2 over both walls, sums of squares wall 0 then wall 1); the
// running extremes are an inclusive scan over the steps (max and min are exact in any
// order) and the time integrals are added one step after another, so that the sums do
// not depend on how the steps were split between flushes.
// acc: [0] int peak tau^2, [1] int sum tau^2, [2 + 2q + w] running extreme q
// (tau max, tau min, p max, p min) of wall w, [10] tangent of int sum tau^2.
__device__ void wall_integrate_body(const WallFlush& f, int nsteps) {
    constexpr int V = kWallAccVals;
    __shared__ double sh[V][kWallThreads];
    const int t = threadIdx.x;
    const int64_t first_step = (int64_t)f.acc[kAccNextStep];
    // per value: 0 sum, 1 max, 2 min
    auto kind = [](int q) { return (q == 0 || q == 1 || q == 10) ? 0 : ((q - 2) / 2 % 2 == 0 ? 1 : 2); };
    double v[V], prev[V];
    lbm_stress_summary sm;
    if (t < nsteps) {
        sm.step = first_step + t;
        double pk = 0.0, s2 = 0.0, ds2 = 0.0;
        for (int w = 0; w < 2; ++w) {
            const double* r = f.scratch + ((long long)t * 2 + w) * kWallPartVals;
            sm.tau_max[w] = r[0]; sm.tau_min[w] = r[2]; sm.p_max[w] = r[4]; sm.p_min[w] = r[6];
            sm.x_tau_max[w] = int32_t(r[1]); sm.x_tau_min[w] = int32_t(r[3]);
            sm.x_p_max[w] = int32_t(r[5]); sm.x_p_min[w] = int32_t(r[7]);
            pk = fmax(pk, fmax(r[0] * r[0], r[2] * r[2]));
            s2 += r[8];
            ds2 += r[9];
        }
        sm.sum_tau2 = s2;
        sm.d_sum_tau2 = ds2;
        v[0] = pk;
        v[1] = s2;
        for (int w = 0; w < 2; ++w) {
            v[2 + w] = sm.tau_max[w];
            v[4 + w] = sm.tau_min[w];
            v[6 + w] = sm.p_max[w];
            v[8 + w] = sm.p_min[w];
        }
        v[10] = ds2;
    } else {
        for (int q = 0; q < V; ++q) v[q] = kind(q) == 0 ? 0.0 : (kind(q) == 1 ? -INFINITY : INFINITY);
    }
    for (int q = 0; q < V; ++q) {
        prev[q] = f.acc[q];
        sh[q][t] = v[q];
    }
    __syncthreads();
    for (int off = 1; off < kWallThreads; off <<= 1) {
        double o[V];
        for (int q = 0; q < V; ++q) o[q] = t >= off ? sh[q][t - off] : 0.0;
        __syncthreads();
        if (t >= off)
            for (int q = 0; q < V; ++q) {
                const int kq = kind(q);
                if (kq == 0) continue;
                v[q] = kq == 1 ? fmax(o[q], v[q]) : fmin(o[q], v[q]);
                sh[q][t] = v[q];
            }
        __syncthreads();
    }
    if (t == 0) {
        double s0 = prev[0], s1 = prev[1], s10 = prev[10];
        for (int k = 0; k < nsteps; ++k) {
            s0 += sh[0][k];
            s1 += sh[1][k];
            s10 += sh[10][k];
            sh[0][k] = s0;
            sh[1][k] = s1;
            sh[10][k] = s10;
        }
    }
    __syncthreads();
    if (t >= nsteps) return;
    double tot[V];
    for (int q = 0; q < V; ++q) {
        const int kq = kind(q);
        tot[q] = kq == 0 ? sh[q][t] : (kq == 1 ? fmax(prev[q], v[q]) : fmin(prev[q], v[q]));
    }
    sm.int_peak_tau2 = tot[0];
    sm.int_tau2 = tot[1];
    sm.d_int_tau2 = tot[10];
    for (int w = 0; w < 2; ++w) {
        sm.run_tau_max[w] = tot[2 + w];
        sm.run_tau_min[w] = tot[4 + w];
        sm.run_p_max[w] = tot[6 + w];
        sm.run_p_min[w] = tot[8 + w];
    }
    f.hist[(sm.step - 1) % f.hist_cap] = sm;
    if (t == nsteps - 1) {
        for (int q = 0; q < V; ++q) f.acc[q] = tot[q];
        f.acc[kAccNextStep] = double(first_step + nsteps);
    }
}

// One lattice, one launch: a block per (wall, step); the last block to finish
// integrates over the steps, then clears the ticket.
__global__ __launch_bounds__(kWallThreads) void wall_flush_kernel(const WallFlush f, int nsteps) {
    __shared__ int last;
    wall_step_reduce(f, blockIdx.y, blockIdx.x);
    if (threadIdx.x == 0) {
        __threadfence();  // this block's values before its ticket
        const unsigned total = gridDim.x * gridDim.y;
        last = atomicAdd(reinterpret_cast<unsigned*>(f.acc + kAccTicket), 1u) == total - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();  // every other block's values after their tickets
    wall_integrate_body(f, nsteps);
    if (threadIdx.x == 0) atomicExch(reinterpret_cast<unsigned*>(f.acc + kAccTicket), 0u);
}

// Many lattices stepped together (same steps), in two launches with the same
// arithmetic: blockIdx.x / 2 (reduction) or blockIdx.x (integration) is the case.
__global__ __launch_bounds__(kWallThreads) void wall_step_reduce_batch_kernel(const WallFlush* __restrict__ tbl) {
    wall_step_reduce(tbl[blockIdx.x >> 1], blockIdx.y, blockIdx.x & 1);
}
__global__ __launch_bounds__(kWallThreads) void wall_integrate_batch_kernel(const WallFlush* __restrict__ tbl,
                                                                            int nsteps) {
    wall_integrate_body(tbl[blockIdx.x], nsteps);
}

}  // namespace

hipError_t launch_step2(const StepArgs& a, int storage, int eos, bool emit, hipStream_t s) {
    switch (storage) {
        case LBM_F64: return launch_step2_f64(a, eos, emit, s);
        case LBM_F32: return launch_step2_f32(a, eos, emit, s);
        case LBM_F16S: return launch_step2_f16s(a, eos, emit, s);
        case LBM_BF16S: return launch_step2_bf16s(a, eos, emit, s);
        case LBM_F32D: return launch_step2_f32d(a, eos, emit, s);
        case LBM_F32S: return launch_step2_f32s(a, eos, emit, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step2_batch(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, int parity,
                              int slot, int storage, int eos, bool emit, hipStream_t s) {
    if (ncases < 1 || total_tiles < 1) return hipErrorInvalidValue;
    switch (storage) {
        case LBM_F64: return launch_batch2_f64(cases, tile_start, ncases, total_tiles, parity, slot, eos, emit, s);
        case LBM_F32: return launch_batch2_f32(cases, tile_start, ncases, total_tiles, parity, slot, eos, emit, s);
        case LBM_F16S: return launch_batch2_f16s(cases, tile_start, ncases, total_tiles, parity, slot, eos, emit, s);
        case LBM_BF16S: return launch_batch2_bf16s(cases, tile_start, ncases, total_tiles, parity, slot, eos, emit, s);
        case LBM_F32D: return launch_batch2_f32d(cases, tile_start, ncases, total_tiles, parity, slot, eos, emit, s);
        case LBM_F32S: return launch_batch2_f32s(cases, tile_start, ncases, total_tiles, parity, slot, eos, emit, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(const StepArgs& a, int storage, int eos, bool emit, hipStream_t s) {
    switch (storage) {
        case LBM_F64: return launch_step_f64(a, eos, emit, s);
        case LBM_F32: return launch_step_f32(a, eos, emit, s);
        case LBM_F16S: return launch_step_f16s(a, eos, emit, s);
        case LBM_BF16S: return launch_step_bf16s(a, eos, emit, s);
        case LBM_F32D: return launch_step_f32d(a, eos, emit, s);
        case LBM_F32S: return launch_step_f32s(a, eos, emit, s);
        case LBM_F64T: return launch_step_f64t(a, eos, emit, s);
        case LBM_F16R: return launch_step_f16r(a, eos, emit, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_batch(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, int parity,
                             int slot, int storage, int eos, int ty, int waves, bool emit, hipStream_t s) {
    if (ncases < 1 || total_tiles < 1) return hipErrorInvalidValue;
    switch (storage) {
        case LBM_F64: return launch_batch_f64(cases, tile_start, ncases, total_tiles, parity, slot, eos, ty, waves, emit, s);
        case LBM_F32: return launch_batch_f32(cases, tile_start, ncases, total_tiles, parity, slot, eos, ty, waves, emit, s);
        case LBM_F16S: return launch_batch_f16s(cases, tile_start, ncases, total_tiles, parity, slot, eos, ty, waves, emit, s);
        case LBM_BF16S: return launch_batch_bf16s(cases, tile_start, ncases, total_tiles, parity, slot, eos, ty, waves, emit, s);
        case LBM_F32D: return launch_batch_f32d(cases, tile_start, ncases, total_tiles, parity, slot, eos, ty, waves, emit, s);
        case LBM_F32S: return launch_batch_f32s(cases, tile_start, ncases, total_tiles, parity, slot, eos, ty, waves, emit, s);
        case LBM_F16R: return launch_batch_f16r(cases, tile_start, ncases, total_tiles, parity, slot, eos, ty, waves, emit, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t pipe_grid(int storage, int eos, int ty, int waves, int* blocks) {
    switch (storage) {
        case LBM_F64: return pipe_grid_f64(eos, ty, waves, blocks);
        case LBM_F32: return pipe_grid_f32(eos, ty, waves, blocks);
        case LBM_F16S: return pipe_grid_f16s(eos, ty, waves, blocks);
        case LBM_BF16S: return pipe_grid_bf16s(eos, ty, waves, blocks);
        case LBM_F32D: return pipe_grid_f32d(eos, ty, waves, blocks);
        case LBM_F32S: return pipe_grid_f32s(eos, ty, waves, blocks);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(const double* rho, void* f, int nx, int ny, int pitch, long long plane, int storage,
                       double q, hipStream_t s) {
    const long long n = (long long)nx * ny;
    const int blocks = int((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    switch (storage) {
        case LBM_F64: hipLaunchKernelGGL(init_kernel<CodecF64>, dim3(blocks), dim3(256), 0, s, rho, f, nx, ny, pitch, plane, q); break;
        case LBM_F32: hipLaunchKernelGGL(init_kernel<CodecF32>, dim3(blocks), dim3(256), 0, s, rho, f, nx, ny, pitch, plane, q); break;
        case LBM_F16S: hipLaunchKernelGGL(init_kernel<CodecF16S>, dim3(blocks), dim3(256), 0, s, rho, f, nx, ny, pitch, plane, q); break;
        case LBM_BF16S: hipLaunchKernelGGL(init_kernel<CodecBF16S>, dim3(blocks), dim3(256), 0, s, rho, f, nx, ny, pitch, plane, q); break;
        case LBM_F32D: hipLaunchKernelGGL(init_kernel<CodecF32D>, dim3(blocks), dim3(256), 0, s, rho, f, nx, ny, pitch, plane, q); break;
        case LBM_F32S: hipLaunchKernelGGL(init_kernel<CodecF32S>, dim3(blocks), dim3(256), 0, s, rho, f, nx, ny, pitch, plane, q); break;
        case LBM_F64T: hipLaunchKernelGGL(init_kernel<CodecF64T>, dim3(blocks), dim3(256), 0, s, rho, f, nx, ny, pitch, plane, q); break;
        case LBM_F16R: hipLaunchKernelGGL(init_kernel<CodecF16R>, dim3(blocks), dim3(256), 0, s, rho, f, nx, ny, pitch, plane, q); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_to_f32(const double* in, float* out, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int blocks = int((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048);
    hipLaunchKernelGGL(to_f32_kernel, dim3(blocks), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, double v, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int blocks = int((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048);
    hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_field_reduce(const double* rho, const double* vx, const double* vy, long long n, double* partials,
                               int nblocks, double* out, hipStream_t s) {
    hipLaunchKernelGGL(field_reduce_stage1, dim3(nblocks), dim3(kRedThreads), 0, s, rho, vx, vy, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(field_reduce_stage2, dim3(1), dim3(kRedThreads), 0, s, partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_column_scan(const double* rho, int nx, int ny, double* colmin, double* centre, hipStream_t s) {
    hipLaunchKernelGGL(column_scan_kernel, dim3((nx + 63) / 64), dim3(64 * kColScanWaves), 0, s, rho, nx, ny, colmin,
                       centre);
    return hipGetLastError();
}

hipError_t launch_wall_reduce(const double* ring, int nsteps, int nx, lbm_stress_summary* hist, int hist_cap,
                              double* scratch, double* acc, hipStream_t s) {
    if (nsteps <= 0) return hipSuccess;
    if (nsteps > kWallThreads) return hipErrorInvalidValue;
    const WallFlush f{ring, nx, hist, hist_cap, scratch, acc};
    hipLaunchKernelGGL(wall_flush_kernel, dim3(2, nsteps), dim3(kWallThreads), 0, s, f, nsteps);
    return hipGetLastError();
}

hipError_t launch_wall_reduce_batch(const WallFlush* tbl, int ncases, int nsteps, hipStream_t s) {
    if (nsteps <= 0 || ncases <= 0) return hipSuccess;
    if (nsteps > kWallThreads || ncases > (1 << 30)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(wall_step_reduce_batch_kernel, dim3(2 * ncases, nsteps), dim3(kWallThreads), 0, s, tbl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(wall_integrate_batch_kernel, dim3(ncases), dim3(kWallThreads), 0, s, tbl, nsteps);
    return hipGetLastError();
}

}  // namespace lbm
