// lbm_noalloc.hip -- the stability/interface check of lbm_check_state_noalloc,
// whose device scratch is a static array of the library instead of memory the
// library or the caller allocates.
//
// The check reduces the emitted fields (mass, momentum, |v|max, NaN count) and
// finds the plug interfaces on the centreline and the liquid columns (Figs. 4a
// and 7a; rupture, Sec. 3.1).  lbm_check_state stages its results in the bound
// workspace and a pinned host buffer the library allocates on the first check;
// this variant keeps its reduction partials, column scans and interface summary
// in `scratch` below and reads back nine doubles, so it allocates nothing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lbm_internal.hpp"

namespace lbm {
namespace {

// Layout of the scratch array (doubles): the reduction partials of
// kFieldReduceBlocks blocks, the five reduced values, the four interface values,
// then the per-column minima and centreline densities of up to kNoAllocMaxNx columns.
constexpr long long kOffPartials = 0;
constexpr long long kOffResult = kOffPartials + 5LL * kFieldReduceBlocks;  // 5 reduced values, 4 interface values
constexpr long long kOffColmin = kOffResult + 32;                          // 256-byte aligned
constexpr long long kOffCentre = kOffColmin + kNoAllocMaxNx;
constexpr long long kScratchDoubles = kOffCentre + kNoAllocMaxNx;
static_assert(kOffColmin % 32 == 0 && kOffCentre % 32 == 0, "sub-buffers 256-byte aligned");

static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` per device, resolved once per device with that device current.
constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

constexpr int kSumThreads = 256;

// Interfaces on the centreline and the liquid columns, from the column scan: a
// column is liquid on the centreline when centre[x] > mid; a run starts at x
// when x is liquid and x - 1 is not (or x = 0).  out: [0] runs, [1] first start,
// [2] last end, [3] liquid columns (colmin[x] > mid), [4] x_rear, [5] x_front
// (NaN unless there is exactly one run and it touches neither end).
__global__ __launch_bounds__(kSumThreads) void interface_summary_kernel(const double* __restrict__ colmin,
                                                                        const double* __restrict__ centre, int nx,
                                                                        double mid, double* __restrict__ out) {
    __shared__ long long sh[3][kSumThreads];
    long long runs = 0, cols = 0, first = nx, last = -1;
    for (int x = threadIdx.x; x < nx; x += kSumThreads) {
        const bool liq = centre[x] > mid;
        const bool prev = x > 0 && centre[x - 1] > mid;
        const bool next = x + 1 < nx && centre[x + 1] > mid;
        if (liq && !prev) {
            ++runs;
            first = min(first, (long long)x);
        }
        if (liq && !next) last = max(last, (long long)x);
        cols += colmin[x] > mid ? 1 : 0;
    }
    sh[0][threadIdx.x] = runs + (cols << 32);
    sh[1][threadIdx.x] = first;
    sh[2][threadIdx.x] = last;
    __syncthreads();
    for (int off = kSumThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + off];
            sh[1][threadIdx.x] = min(sh[1][threadIdx.x], sh[1][threadIdx.x + off]);
            sh[2][threadIdx.x] = max(sh[2][threadIdx.x], sh[2][threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const long long nruns = sh[0][0] & 0xFFFFFFFFLL, ncols = sh[0][0] >> 32;
    const long long f = sh[1][0], l = sh[2][0];
    out[0] = double(nruns);
    out[1] = double(f);
    out[2] = double(l);
    out[3] = double(ncols);
    double xr = __builtin_nan(""), xf = __builtin_nan("");
    if (nruns == 1 && f > 0 && l < nx - 1) {
        xr = (f - 1) + (mid - centre[f - 1]) / (centre[f] - centre[f - 1]);
        xf = l + (centre[l] - mid) / (centre[l] - centre[l + 1]);
    }
    out[4] = xr;
    out[5] = xf;
}

}  // namespace

hipError_t noalloc_setup() {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double*>(p);
    return hipSuccess;
}

hipError_t noalloc_check(int device, const double* rho, const double* vx, const double* vy, int nx, int ny,
                         double mid, double* host9, hipStream_t s) {
    if (nx < 1 || nx > kNoAllocMaxNx || ny < 1) return hipErrorInvalidValue;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    double* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = g_scratch[device];
    }
    if (!base) return hipErrorNotInitialized;
    hipError_t e = launch_field_reduce(rho, vx, vy, (long long)nx * ny, base + kOffPartials, kFieldReduceBlocks,
                                       base + kOffResult, s);
    if (e != hipSuccess) return e;
    e = launch_column_scan(rho, nx, ny, base + kOffColmin, base + kOffCentre, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(interface_summary_kernel, dim3(1), dim3(kSumThreads), 0, s, base + kOffColmin,
                       base + kOffCentre, nx, mid, base + kOffResult + 5);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the five reduced values and four of the interface values: runs are not needed on the host
    double res[11];
    e = hipMemcpyAsync(res, base + kOffResult, sizeof res, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (int q = 0; q < 5; ++q) host9[q] = res[q];
    host9[5] = res[8];   // liquid columns
    host9[6] = res[9];   // x_rear
    host9[7] = res[10];  // x_front
    host9[8] = res[5];   // runs
    return hipSuccess;
}

}  // namespace lbm
