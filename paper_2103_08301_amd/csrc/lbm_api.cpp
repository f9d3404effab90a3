// lbm_api.cpp -- host side of the C ABI declared in include/lbm.h.
//
// Parameter validation, the equation of state (critical point and Maxwell
// coexistence, paper Sec. 2.2 "Verification"), the plug initial condition
// (Sec. 2.3 / 3.1), the layout of the caller-owned device workspace, and the
// launch sequence of lbm_step.  All per-node work runs in lbm_kernels.hip.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.hpp"

namespace {

// ---------------------------------------------------------------------------
// Second-order forward-mode automatic differentiation: value, d/drho, d2/drho2.

struct Dual2 {
    double v, d, dd;
};
inline Dual2 operator+(Dual2 a, Dual2 b) { return {a.v + b.v, a.d + b.d, a.dd + b.dd}; }
inline Dual2 operator-(Dual2 a, Dual2 b) { return {a.v - b.v, a.d - b.d, a.dd - b.dd}; }
inline Dual2 operator*(Dual2 a, Dual2 b) { return {a.v * b.v, a.d * b.v + a.v * b.d, a.dd * b.v + 2 * a.d * b.d + a.v * b.dd}; }
inline Dual2 operator*(double s, Dual2 a) { return {s * a.v, s * a.d, s * a.dd}; }
inline Dual2 operator+(double s, Dual2 a) { return {s + a.v, a.d, a.dd}; }
inline Dual2 operator-(double s, Dual2 a) { return {s - a.v, -a.d, -a.dd}; }
inline Dual2 recip(Dual2 a) {
    const double r = 1.0 / a.v;
    return {r, -a.d * r * r, (2 * a.d * a.d * r - a.dd) * r * r};
}
inline Dual2 operator/(Dual2 a, Dual2 b) { return a * recip(b); }

// p0 = RT * rep(rho) - aA * att(rho)
struct Eos {
    int kind;
    double a, b, R;
    double Tc, T, alpha;

    Dual2 rep(Dual2 r) const {
        if (kind == LBM_EOS_CS) {
            const Dual2 h = (0.25 * b) * r;
            const Dual2 om = 1.0 - h;
            return r * (1.0 + h * (1.0 + h * (1.0 - h))) / (om * om * om);
        }
        return r / (1.0 - b * r);
    }
    Dual2 att(Dual2 r) const {
        if (kind == LBM_EOS_CS) return r * r;
        return r * r / (1.0 + b * r * (2.0 - b * r));
    }
    double rho_max() const { return kind == LBM_EOS_CS ? 4.0 / b : 1.0 / b; }
    Dual2 p(double rho) const {
        const Dual2 r{rho, 1.0, 0.0};
        return (R * T) * rep(r) - (a * alpha) * att(r);
    }
};

double pr_alpha(double omega, double T, double Tc) {
    const double kw = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
    const double s = 1.0 + kw * (1.0 - std::sqrt(T / Tc));
    return s * s;
}

// d alpha / dT at fixed Tc.
double pr_alpha_dT(double omega, double T, double Tc) {
    const double kw = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
    const double s = 1.0 + kw * (1.0 - std::sqrt(T / Tc));
    return -kw * s / std::sqrt(T * Tc);
}

// Critical point: p' = p'' = 0.  With p = T A(rho) + B(rho) (alpha(Tc) = 1),
// T = -B'/A' and the density solves A' B'' - A'' B' = 0.
bool critical_point(Eos& e, double& rho_c) {
    auto cond = [&](double rho) {
        const Dual2 r{rho, 1.0, 0.0};
        const Dual2 A = e.R * e.rep(r);
        const Dual2 B = -e.a * e.att(r);
        return A.d * B.dd - A.dd * B.d;
    };
    const double rmax = e.rho_max();
    double lo = rmax * 1e-6, flo = cond(lo), hi = 0;
    bool found = false;
    for (int k = 1; k <= 4000; ++k) {  // geometric scan up to the excluded-volume limit
        const double r = rmax * 1e-6 * std::pow(1e6 * 0.999, k / 4000.0);
        const double fr = cond(r);
        if ((flo > 0) != (fr > 0)) { hi = r; found = true; break; }
        lo = r;
        flo = fr;
    }
    if (!found) return false;
    for (int it = 0; it < 200 && hi - lo > 4 * std::numeric_limits<double>::epsilon() * hi; ++it) {
        const double m = 0.5 * (lo + hi), fm = cond(m);
        if ((fm > 0) == (flo > 0)) { lo = m; flo = fm; } else { hi = m; }
    }
    rho_c = 0.5 * (lo + hi);
    const Dual2 r{rho_c, 1.0, 0.0};
    e.Tc = -(-e.a * e.att(r)).d / (e.R * e.rep(r)).d;
    return true;
}

// chemical potential difference mu(rl) - mu(rg) = int p'(rho)/rho drho
// = int_{ln rg}^{ln rl} p'(e^s) ds, by Romberg integration (at most 2^15 + 1
// evaluations; the integrand is analytic in s).
double dmu(const Eos& e, double rg, double rl, double scale) {
    const double a = std::log(rg), b = std::log(rl);
    auto f = [&](double s) { return e.p(std::exp(s)).d; };
    constexpr int kLevels = 16;
    double R[kLevels][kLevels];
    double h = b - a;
    R[0][0] = 0.5 * h * (f(a) + f(b));
    for (int k = 1; k < kLevels; ++k) {
        h *= 0.5;
        double sum = 0.0;
        const long n = 1L << (k - 1);
        for (long j = 0; j < n; ++j) sum += f(a + (2 * j + 1) * h);
        R[k][0] = 0.5 * R[k - 1][0] + h * sum;
        double pow4 = 1.0;
        for (int m = 1; m <= k; ++m) {
            pow4 *= 4.0;
            R[k][m] = R[k][m - 1] + (R[k][m - 1] - R[k - 1][m - 1]) / (pow4 - 1.0);
        }
        if (k >= 5 && std::fabs(R[k][k] - R[k - 1][k - 1]) <= 1e-15 * (std::fabs(R[k][k]) + scale)) return R[k][k];
    }
    return R[kLevels - 1][kLevels - 1];
}

// Coexistence at temperature e.T: the pressure p* at which the gas and liquid
// roots of p0(rho) = p* (one on each stable branch) have equal chemical
// potential, mu(rho_l) - mu(rho_g) = int p'(rho)/rho drho = 0.  The difference
// decreases monotonically in p*, so p* is bracketed between the spinodal
// pressures and bisected (geometrically while the bracket spans decades).
struct Coexist {
    static double branch_root(const Eos& e, double target, double lo, double hi) {
        for (int it = 0; it < 300; ++it) {  // p0 increases on [lo, hi]
            const double m = 0.5 * (lo + hi);
            if (!(m > lo && m < hi)) break;
            (e.p(m).v < target ? lo : hi) = m;
        }
        return 0.5 * (lo + hi);
    }

    static bool solve(const Eos& base, double T, double omega, double& rho_g, double& rho_l) {
        Eos e = base;
        e.T = T;
        e.alpha = (e.kind == LBM_EOS_PR) ? pr_alpha(omega, T, e.Tc) : 1.0;
        const double rmax = e.rho_max();
        auto dp = [&](double r) { return e.p(r).d; };
        // spinodals: first sign changes of p' on a geometric grid
        constexpr int kGrid = 40000;
        double sg = -1, sl = -1, prev = rmax * 1e-12;
        bool in_unstable = false;
        for (int k = 1; k <= kGrid; ++k) {
            const double r = rmax * 1e-12 * std::pow(1e12 * (1 - 1e-9), double(k) / kGrid);
            const double d = dp(r);
            if (!in_unstable && d < 0) {
                double lo = prev, hi = r;
                for (int it = 0; it < 200; ++it) { const double m = 0.5 * (lo + hi); (dp(m) > 0 ? lo : hi) = m; }
                sg = lo;
                in_unstable = true;
            } else if (in_unstable && d > 0) {
                double lo = prev, hi = r;
                for (int it = 0; it < 200; ++it) { const double m = 0.5 * (lo + hi); (dp(m) < 0 ? lo : hi) = m; }
                sl = hi;
                break;
            }
            prev = r;
        }
        if (sg < 0 || sl < 0) return false;
        double p_hi = e.p(sg).v, p_lo = e.p(sl).v;
        if (!(p_lo > 0)) p_lo = p_hi * 1e-300;
        double g = 0, l = 0;
        for (int it = 0; it < 3000; ++it) {
            const double pm = (p_hi > 4 * p_lo) ? std::sqrt(p_lo * p_hi) : 0.5 * (p_lo + p_hi);
            if (!(pm > p_lo && pm < p_hi)) break;
            g = branch_root(e, pm, 0.0, sg);
            l = branch_root(e, pm, sl, rmax);
            (dmu(e, g, l, e.R * e.T) > 0 ? p_lo : p_hi) = pm;
        }
        const double ps = 0.5 * (p_lo + p_hi);
        rho_g = branch_root(e, ps, 0.0, sg);
        rho_l = branch_root(e, ps, sl, rmax);
        return std::isfinite(rho_g) && std::isfinite(rho_l) && rho_g > 0 && rho_g < rho_l && rho_l < rmax;
    }
};

// SplitMix64 (Steele, Lea & Flood 2014): the n-th output (0-based) of the
// generator seeded with `seed`.
uint64_t splitmix64_nth(uint64_t seed, uint64_t n) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (n + 1);
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

size_t storage_bytes(int storage) {
    switch (storage) {
        case LBM_F64T: return 16;
        case LBM_F64: return 8;
        case LBM_F32:
        case LBM_F32D:
        case LBM_F32S: return 4;
        default: return 2;
    }
}

constexpr int kRingCap = 256;  // per-step wall-ring slots before a wall reduction is forced
constexpr int kDefaultMarchRows = 16;

// Tile heights each schedule is compiled for (0 picks the default).
bool schedule_ok(const lbm_params* p) {
    const int r = p->tile_rows, w = p->tile_waves;
    if (w != 0 && w != 4 && w != 8) return false;
    if (p->pipe_blocks != 0 && (p->schedule != lbm::kSchedulePipe || p->pipe_blocks < 8)) return false;
    if (p->storage == LBM_F16R && p->schedule != lbm::kScheduleTile) return false;  // stochastic rounding: tiles only
    if (p->storage == LBM_F64T)  // tangent-linear runs: the tile schedule with 12-row, 8-wave tiles
        return p->schedule == lbm::kScheduleTile && (r == 0 || r == 12) && (w == 0 || w == 8);
    switch (p->schedule) {
        case lbm::kScheduleTile:
            if (w == 8) return r == 0 || r == 12 || r == 20 || r == 28;
            return r == 0 || r == 8 || r == 12 || r == 20 || r == 28;
        case lbm::kScheduleMarch: return w == 0 && (r == 0 || (r >= 4 && r <= 256));
        case lbm::kSchedulePipe:
            if (w == 8) return r == 0 || r == 8 || r == 16;
            return r == 0 || r == 4 || r == 8 || r == 12;
        default: return false;
    }
}

bool graph_steps_ok(int g) {
    return g == -1 || g == 0 || g == 2 || g == 4 || g == 8 || g == 16 || g == 32 || g == 64 || g == 128 || g == 256;
}

// Captured HIP graphs of consecutive step launches, made when first needed:
// replaying a graph issues its launches without a host call per kernel.  Runs
// of the full graph length are kept per (parity of the input buffer, first
// wall-ring slot); shorter runs, and the last run of a call, which ends with the
// wall flush of the ring so far, per (parity, first slot, length, flush), up to
// kMaxShortGraphs of them, beyond which such runs are launched kernel by kernel.
// The graphs hold only step and flush kernels (no memset nodes).
constexpr size_t kMaxShortGraphs = 64;
struct StepGraphs {
    hipStream_t cap = nullptr;  // private capture stream (default priority)
    hipGraphExec_t exec[2][kRingCap] = {};
    std::map<uint32_t, hipGraphExec_t> shorter;  // key: (length << 10) | (flush << 9) | (slot << 1) | parity
    // The cache entry for a run of `len` steps from (parity, slot), followed by the
    // wall flush if `flush`, or null when the cache of other runs is full and the run
    // must be launched kernel by kernel.
    hipGraphExec_t* entry(int parity, int slot, int len, int full_len, bool flush) {
        if (len == full_len && !flush) return &exec[parity][slot];
        const uint32_t key = ((uint32_t)len << 10) | ((uint32_t)flush << 9) | ((uint32_t)slot << 1) | (uint32_t)parity;
        auto it = shorter.find(key);
        if (it != shorter.end()) return &it->second;
        if (shorter.size() >= kMaxShortGraphs) return nullptr;
        return &shorter.emplace(key, nullptr).first->second;
    }
    void drop() {
        for (auto& row : exec)
            for (auto& e : row)
                if (e) { (void)hipGraphExecDestroy(e); e = nullptr; }
        for (auto& kv : shorter)
            if (kv.second) (void)hipGraphExecDestroy(kv.second);
        shorter.clear();
    }
    ~StepGraphs() {
        drop();
        if (cap) (void)hipStreamDestroy(cap);
    }
};

// Captures `steps` launches made by launch(k) (k = 0 .. steps-1) into one executable graph.
template <class F>
hipError_t capture_graph(StepGraphs& g, int steps, F&& launch, hipGraphExec_t* out) {
    hipError_t e = hipSuccess;
    if (!g.cap) e = hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int k = 0; k < steps && le == hipSuccess; ++k) le = launch(k, g.cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(g.cap, &graph);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    return e;
}

}  // namespace

struct lbm_ctx {
    double* check_host = nullptr;  // pinned host copy of a check's device results: 5 sums, colmin[nx], centre[nx]
    ~lbm_ctx() {
        if (check_host) (void)hipHostFree(check_host);
    }
    int nx = 0, ny = 0;
    double tau = 1.0;
    lbm_params p{};
    Eos eos{};
    double rho_c = 0, rho_g = NAN, rho_l = NAN, rho_w = 0;
    double shift_q = 0;  // shifted storage: f_i - 9 w_i q is stored, q = rho0_shift / 9 on a 2^-24 grid
    int pitch = 0;
    long long plane = 0;
    int nstrip = 0, nchunk = 0, ty = 0, schedule = 0, tile_waves = 4, pipe_blocks = 0;
    // workspace layout (byte offsets)
    size_t off_f[2]{}, off_rho = 0, off_vx = 0, off_vy = 0, off_ring = 0, off_hist = 0,
           off_acc = 0, off_wscr = 0, off_red = 0, off_redout = 0, off_colmin = 0, off_centre = 0, off_tickets = 0,
           off_sr = 0, total = 0;
    char* dev = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    bool bound = false, initialized = false;
    bool in_batch = false;  // owned by an lbm_batch: stepped only through lbm_batch_step
    double dtheta[4] = {0, 0, 0, 0};  // F64T: tangent direction (dp, a, b, T)
    // reverse-mode sensitivities (lbm_adjoint_*): a second caller-owned workspace
    struct Adjoint {
        char* dev = nullptr;
        bool bound = false, recorded = false, swept = false;
        int64_t n = 0, seg = 0, nckpt = 0;  // recorded steps, segment length, checkpoints
        size_t state = 0, lam = 0, fld = 0;  // bytes of one state / adjoint field / step's forward fields (aligned)
        size_t off_ckpt = 0, off_pp = 0, off_fld = 0, off_lam[2]{}, off_tw = 0, off_part = 0, off_red = 0,
               off_acc = 0, off_pw = 0, off_g0 = 0, total = 0;
        int blocks = 0, cur = 0, ty = 8, waves = 4, ring_cap = 0;
        int objective = LBM_J_SUM_TAU2;
        size_t off_seed = 0;  // peak objective: dJ/dtau_w of each step of two segments
        double J = 0, seed = 1;
        // captured graphs of a full segment: its recompute into field buffer b, and its adjoint
        // sweep (with the reduction) reading buffer b at adjoint parity p
        hipGraphExec_t rec_graph[2] = {nullptr, nullptr}, adj_graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
        // the recompute of the next segment runs on its own stream beside the current adjoint sweep
        hipStream_t aux = nullptr;
        hipEvent_t ev_start = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_adj[2] = {nullptr, nullptr};
        void drop_graphs() {
            for (auto& g : rec_graph)
                if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
            for (auto& row : adj_graph)
                for (auto& g : row)
                    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
        }
        ~Adjoint() {
            drop_graphs();
            for (hipEvent_t e : {ev_start, ev_rec[0], ev_rec[1], ev_adj[0], ev_adj[1]})
                if (e) (void)hipEventDestroy(e);
            if (aux) (void)hipStreamDestroy(aux);
        }
        Adjoint() = default;
        Adjoint& operator=(const Adjoint& o) {  // layout only; graphs, stream and events stay with this one
            drop_graphs();
            dev = o.dev; bound = o.bound; recorded = o.recorded; swept = o.swept;
            n = o.n; seg = o.seg; nckpt = o.nckpt; state = o.state; lam = o.lam; fld = o.fld;
            off_ckpt = o.off_ckpt; off_pp = o.off_pp; off_fld = o.off_fld;
            off_lam[0] = o.off_lam[0]; off_lam[1] = o.off_lam[1];
            off_tw = o.off_tw; off_part = o.off_part; off_red = o.off_red; off_acc = o.off_acc; off_pw = o.off_pw;
            off_g0 = o.off_g0; total = o.total; blocks = o.blocks; cur = o.cur; ty = o.ty; waves = o.waves;
            ring_cap = o.ring_cap;
            objective = o.objective; off_seed = o.off_seed;
            J = o.J; seed = o.seed;
            return *this;
        }
        Adjoint(const Adjoint&) = delete;
    } adj;
    int cur = 0;
    int64_t steps = 0;
    // Step whose density and velocity the field buffers hold.  A call of lbm_step emits them only
    // at a check; the fields of a later step are made when asked for, by running that step again
    // with field output from its input, which the other distribution buffer still holds while
    // prev_valid (the run gives the same distributions, wall arrays and step counter words).
    int64_t fields_step = 0;
    bool prev_valid = false;
    int ring_fill = 0;
    int last_slot = -1;  // wall-ring slot of the latest step (its wall arrays)
    int64_t ring_first_step = 1;
    int64_t hist_first = 1;  // first step whose summary is in the history ring (after lbm_load: the next step)
    lbm_check_result check{};
    std::string err;
    StepGraphs graphs;  // captured step loops (invalidated when the launch arguments change)
    int graph_steps() const {
        if (p.graph_steps < 0 || schedule == lbm::kSchedulePipe) return 0;
        return p.graph_steps == 0 ? 64 : p.graph_steps;
    }
    // steps per launch of lbm_step: 2 with the tile schedule's two-step kernel (on request)
    int steps_per_launch() const {
        return (schedule == lbm::kScheduleTile && p.storage != LBM_F64T && p.fused_steps == 2) ? 2 : 1;
    }

    template <class T>
    T* at(size_t off) const { return reinterpret_cast<T*>(dev + off); }
};

namespace {

lbm_status fail(lbm_ctx* c, lbm_status s, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        std::vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

// Whether the first and the last byte of [p, p + bytes) are device memory of the current
// device.  A host pointer handed to a bind call (or as a device output) by mistake would
// otherwise surface only as a memory fault of the first kernel that touches it; this turns
// it into an error before anything is launched.  (Memory of another allocation right after
// the buffer cannot be told apart.)  LBM_OK when the range is usable; LBM_EDEVICE when there
// is no current device, LBM_EINVAL for memory that is not on it, with the reason in *why.
lbm_status device_range_check(const void* p, size_t bytes, const char** why) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        *why = "no current HIP device";
        return LBM_EDEVICE;
    }
    const char* ends[2] = {static_cast<const char*>(p), static_cast<const char*>(p) + (bytes ? bytes - 1 : 0)};
    for (const char* q : ends) {
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, q) != hipSuccess) {
            (void)hipGetLastError();  // clear it, so that the next HIP call does not report it
            *why = "not HIP device memory";
            return LBM_EINVAL;
        }
        if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged) {
            *why = "not HIP device memory (host or unregistered memory)";
            return LBM_EINVAL;
        }
        if (at.device != dev) {
            *why = "memory of another device than the current one";
            return LBM_EINVAL;
        }
    }
    return LBM_OK;
}

#define HIP_TRY(ctx, expr)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(ctx, LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

lbm_status reset_diagnostics(lbm_ctx* c) {
    const long long nxy = (long long)c->nx * c->ny;
    HIP_TRY(c, lbm::launch_fill(c->at<double>(c->off_vx), 0.0, nxy, c->stream));
    HIP_TRY(c, lbm::launch_fill(c->at<double>(c->off_vy), 0.0, nxy, c->stream));
    double* acc = c->at<double>(c->off_acc);
    HIP_TRY(c, lbm::launch_fill(acc, 0.0, 2, c->stream));
    for (int q = 0; q < 4; ++q)  // running maxima start at -inf, minima at +inf
        HIP_TRY(c, lbm::launch_fill(acc + 2 + 2 * q, (q % 2 == 0) ? -INFINITY : INFINITY, 2, c->stream));
    HIP_TRY(c, lbm::launch_fill(acc + 10, 0.0, 1, c->stream));  // tangent of the sum-of-squares integral
    HIP_TRY(c, lbm::launch_fill(acc + lbm::kAccTicket, 0.0, 1, c->stream));  // the wall flush's ticket
    HIP_TRY(c, lbm::launch_fill(acc + lbm::kAccNextStep, 1.0, 1, c->stream));  // the first step to flush
    HIP_TRY(c, lbm::launch_fill(c->at<double>(c->off_sr), 0.0, 1, c->stream));  // stochastic-rounding step counters
    c->steps = 0;
    c->fields_step = 0;  // the initialisation writes the density and zero velocity
    c->prev_valid = false;
    c->ring_fill = 0;
    c->last_slot = -1;
    c->ring_first_step = 1;
    c->hist_first = 1;
    c->check = lbm_check_result{};
    c->check.rupture_step = -1;
    c->check.unstable_step = -1;
    c->check.x_rear = NAN;
    c->check.x_front = NAN;
    return LBM_OK;
}

lbm_status run_check(lbm_ctx* c);

lbm_status init_from_device_rho(lbm_ctx* c) {
    HIP_TRY(c, lbm::launch_init(c->at<double>(c->off_rho), c->dev + c->off_f[0], c->nx, c->ny, c->pitch, c->plane,
                                c->p.storage, c->shift_q, c->stream));
    c->cur = 0;
    lbm_status s = reset_diagnostics(c);
    if (s) return s;
    c->initialized = true;
    return run_check(c);
}

lbm_status flush_wall(lbm_ctx* c) {
    if (c->ring_fill == 0) return LBM_OK;
    if (!c->p.y_periodic) {
        HIP_TRY(c, lbm::launch_wall_reduce(c->at<double>(c->off_ring), c->ring_fill, c->nx,
                                           c->at<lbm_stress_summary>(c->off_hist), c->p.history_cap,
                                           c->at<double>(c->off_wscr), c->at<double>(c->off_acc), c->stream));
    }
    c->ring_first_step += c->ring_fill;
    c->ring_fill = 0;
    return LBM_OK;
}

// A check in two halves, so that a batch can launch every case's before waiting once:
// check_launch queues the reductions of the emitted fields and their copies to the
// pinned host buffer; check_finish (after the stream has been synchronised) derives
// mass, momentum, |v|max, NaNs, interface positions and rupture.
lbm_status check_launch(lbm_ctx* c) {
    if (!c->check_host) {
        void* h = nullptr;
        HIP_TRY(c, hipHostMalloc(&h, (5 + 2 * (size_t)c->nx) * sizeof(double), hipHostMallocDefault));
        c->check_host = static_cast<double*>(h);
    }
    const long long nxy = (long long)c->nx * c->ny;
    HIP_TRY(c, lbm::launch_field_reduce(c->at<double>(c->off_rho), c->at<double>(c->off_vx), c->at<double>(c->off_vy),
                                        nxy, c->at<double>(c->off_red), lbm::kFieldReduceBlocks,
                                        c->at<double>(c->off_redout), c->stream));
    HIP_TRY(c, lbm::launch_column_scan(c->at<double>(c->off_rho), c->nx, c->ny, c->at<double>(c->off_colmin),
                                       c->at<double>(c->off_centre), c->stream));
    double* h = c->check_host;
    HIP_TRY(c, hipMemcpyAsync(h, c->dev + c->off_redout, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(h + 5, c->dev + c->off_colmin, c->nx * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(h + 5 + c->nx, c->dev + c->off_centre, c->nx * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    return LBM_OK;
}

// Fills the check result from the reduced fields (sum rho, sum rho vx, sum rho vy, max |v|^2,
// NaN count) and the centreline interfaces and liquid columns, and detects rupture and
// instability.
lbm_status check_apply(lbm_ctx* c, const double* red, double x_rear, double x_front, int liquid_columns) {
    lbm_check_result& k = c->check;
    k.step = c->steps;
    k.mass = red[0];
    k.momx = red[1];
    k.momy = red[2];
    k.vmax = std::sqrt(red[3]);
    k.nan_count = (int64_t)red[4];
    k.x_rear = x_rear;
    k.x_front = x_front;
    k.liquid_columns = liquid_columns;
    const double mid = 0.5 * (c->rho_g + c->rho_l);
    if (std::isfinite(mid) && c->steps > 0 && k.liquid_columns == 0 && k.rupture_step < 0) k.rupture_step = c->steps;
    const bool bad = k.nan_count > 0 || !(k.vmax <= c->p.v_limit);
    if (bad && k.unstable_step < 0) {
        k.unstable_step = c->steps;
        return fail(c, LBM_EUNSTABLE, "instability at step %lld: nan cells %lld, |v|max %g",
                    (long long)c->steps, (long long)k.nan_count, k.vmax);
    }
    if (bad) return fail(c, LBM_EUNSTABLE, "state is unstable since step %lld", (long long)k.unstable_step);
    return LBM_OK;
}

lbm_status check_finish(lbm_ctx* c) {
    const double* red = c->check_host;
    const double* colmin = red + 5;
    const double* centre = red + 5 + c->nx;
    // interfaces: crossings of the midpoint density on the centreline
    const double mid = 0.5 * (c->rho_g + c->rho_l);
    double x_rear = NAN, x_front = NAN;
    int liquid_columns = 0;
    if (std::isfinite(mid)) {
        int runs = 0, first = -1, last = -1;
        bool prev = false;
        for (int x = 0; x < c->nx; ++x) {
            const bool liq = centre[x] > mid;
            if (liq && !prev) { ++runs; first = x; }
            if (liq) last = x;
            prev = liq;
        }
        if (runs == 1 && first > 0 && last < c->nx - 1) {
            x_rear = (first - 1) + (mid - centre[first - 1]) / (centre[first] - centre[first - 1]);
            x_front = last + (centre[last] - mid) / (centre[last] - centre[last + 1]);
        }
        for (int x = 0; x < c->nx; ++x) liquid_columns += colmin[x] > mid ? 1 : 0;
    }
    return check_apply(c, red, x_rear, x_front, liquid_columns);
}

lbm_status run_check(lbm_ctx* c) {
    lbm_status s = check_launch(c);
    if (s) return s;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return check_finish(c);
}

// Points the wall arrays of a step's arguments at a slot of the wall ring.
void set_wall_slot(lbm::StepArgs& a, const lbm_ctx* c, int slot) {
    double* w = c->at<double>(c->off_ring) + (size_t)slot * lbm::kWallSlotVals * c->nx;
    a.tau_w = w;
    a.p_w = w + 2 * (size_t)c->nx;
    a.dtau_w = w + 4 * (size_t)c->nx;
}

lbm::StepArgs make_args(const lbm_ctx* c) {
    lbm::StepArgs a{};
    a.nx = c->nx;
    a.ny = c->ny;
    a.pitch = c->pitch;
    a.plane = c->plane;
    a.nstrip = c->nstrip;
    a.nchunk = c->nchunk;
    a.ty = c->ty;
    a.schedule = c->schedule;
    a.tile_waves = c->tile_waves;
    a.xper = c->p.x_periodic;
    a.yper = c->p.y_periodic;
    a.tau = c->tau;
    a.s_e = c->p.s_e;
    a.s_eps = c->p.s_eps;
    a.s_q = c->p.s_q;
    a.s_v = 1.0 / c->tau;
    a.s_j = c->p.s_j > 0 ? c->p.s_j : 1.0 / c->tau;
    a.k2 = c->p.k * c->p.k;
    a.kappa = c->p.kappa;
    a.g = c->p.dp / c->nx;
    a.nu = (c->tau - 0.5) / 3.0;
    a.RT = c->eos.R * c->eos.T;
    a.a_eff = c->eos.a * c->eos.alpha;
    a.b = c->eos.b;
    a.rho_w = c->rho_w;
    a.rho0 = c->shift_q;
    a.cf = lbm::CoefF32{float(a.tau), float(a.s_e), float(a.s_eps), float(a.s_q), float(a.s_j), float(a.s_v),
                        float(a.k2), float(a.kappa), float(a.g), float(a.nu), float(a.RT), float(a.a_eff),
                        float(a.b), float(a.rho_w), float(a.rho0)};
    a.ring = c->at<double>(c->off_ring);
    a.rho_out = c->at<double>(c->off_rho);
    a.vx_out = c->at<double>(c->off_vx);
    a.vy_out = c->at<double>(c->off_vy);
    a.ct = lbm::CoefTangent{};
    if (c->p.storage == LBM_F64T) {
        const double dT = c->dtheta[3];
        a.ct.g = c->dtheta[0] / c->nx;
        a.ct.RT = c->eos.R * dT;
        a.ct.a_eff = c->eos.alpha * c->dtheta[1] +
                     (c->p.eos == LBM_EOS_PR ? c->eos.a * pr_alpha_dT(c->p.omega, c->eos.T, c->eos.Tc) * dT : 0.0);
        a.ct.b = c->dtheta[2];
    }
    a.tickets = c->at<unsigned long long>(c->off_tickets);
    a.pipe_blocks = c->pipe_blocks;
    a.sr = c->at<uint32_t>(c->off_sr);
    a.sr_par = c->cur;
    return a;
}

}  // namespace

extern "C" {

void lbm_params_default(lbm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->eos = LBM_EOS_CS;
    p->a = 1.0;
    p->b = 4.0;
    p->R = 1.0;
    p->omega = 0.344;
    p->T_over_Tc = 0.85;
    p->k = 1.0;
    p->kappa = 0.001;
    p->s_e = 1.64;
    p->s_eps = 1.54;
    p->s_q = 1.7;
    p->s_j = 0.0;
    p->rho_wall = NAN;
    p->dp = 0.0;
    p->x_periodic = 0;
    p->y_periodic = 0;
    p->storage = LBM_F32;
    p->rho0_shift = NAN;
    p->check_every = 1000;
    p->v_limit = 0.5;
    p->history_cap = 4096;
    p->tile_rows = 0;
    p->schedule = 0;
    p->tile_waves = 0;
    p->pipe_blocks = 0;
    p->graph_steps = 0;
    p->fused_steps = 0;
}

lbm_status lbm_create(int nx, int ny, double tau, const lbm_params* p, lbm_ctx** out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (!p) return LBM_EINVAL;
    auto rate_ok = [](double s) { return s > 0 && s < 2; };
    if (nx < 4 || ny < 4 || !(tau > 0.5) || !(p->a > 0) || !(p->b > 0) || !(p->R > 0) || !(p->T_over_Tc > 0) ||
        !std::isfinite(p->T_over_Tc) || !(p->k > 0) || !(p->kappa >= 0) || !rate_ok(p->s_e) || !rate_ok(p->s_eps) ||
        !rate_ok(p->s_q) || !(p->s_j <= 0 || rate_ok(p->s_j)) || !std::isfinite(p->dp) || p->check_every < 1 ||
        !(p->v_limit > 0) || p->history_cap < 1 || (p->eos != LBM_EOS_CS && p->eos != LBM_EOS_PR) ||
        p->storage < LBM_F64 || p->storage > LBM_F16R || (p->x_periodic != 0 && p->x_periodic != 1) ||
        (p->y_periodic != 0 && p->y_periodic != 1) || !std::isfinite(p->omega) ||
        (!std::isnan(p->rho_wall) && !(p->rho_wall > 0)) || !schedule_ok(p) || !graph_steps_ok(p->graph_steps) ||
        p->fused_steps < 0 || p->fused_steps > 2 || (p->storage == LBM_F16R && p->fused_steps == 2))
        return LBM_EINVAL;
    const int pitch = (nx + 63) / 64 * 64;
    // the step kernel addresses a distribution buffer with 32-bit byte offsets
    if ((unsigned long long)pitch * ny * 9 * storage_bytes(p->storage) >= (1ULL << 32)) return LBM_EINVAL;
    // the pipelined schedule drops halo-lane stores with a 2 GiB out-of-range buffer offset
    if (p->schedule == lbm::kSchedulePipe && (unsigned long long)pitch * ny * 9 * storage_bytes(p->storage) >= (1ULL << 31))
        return LBM_EINVAL;
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_ENOMEM;
    c->nx = nx;
    c->ny = ny;
    c->tau = tau;
    c->p = *p;
    c->eos.kind = p->eos;
    c->eos.a = p->a;
    c->eos.b = p->b;
    c->eos.R = p->R;
    if (!critical_point(c->eos, c->rho_c)) { delete c; return LBM_EINVAL; }
    c->eos.T = p->T_over_Tc * c->eos.Tc;
    c->eos.alpha = p->eos == LBM_EOS_PR ? pr_alpha(p->omega, c->eos.T, c->eos.Tc) : 1.0;
    if (p->T_over_Tc < 1.0) {
        if (!Coexist::solve(c->eos, c->eos.T, p->omega, c->rho_g, c->rho_l)) { delete c; return LBM_EINVAL; }
    }
    const double liquid = std::isnan(c->rho_l) ? c->rho_c : c->rho_l;
    c->rho_w = std::isnan(p->rho_wall) ? liquid : p->rho_wall;
    const double rho0 = std::isnan(p->rho0_shift) ? (std::isnan(c->rho_g) ? c->rho_c : c->rho_g) : p->rho0_shift;
    // the shift constants 9 w_i q = {4, 1, 1/4} q are then dyadic with few bits (exact in FP32)
    c->shift_q = std::ldexp(std::nearbyint(std::ldexp(rho0 / 9.0, 24)), -24);
    c->pitch = pitch;
    c->plane = (long long)pitch * ny;
    c->nstrip = (nx + lbm::kStripOut - 1) / lbm::kStripOut;
    c->schedule = p->schedule;
    c->tile_waves = p->tile_waves > 0 ? p->tile_waves : (p->storage == LBM_F64T ? 8 : 4);
    // measured on the 4096x512 plug channel: 8-row tiles for FP32/FP16/BF16 arithmetic
    // tiles, 12-row tiles when the arithmetic is FP64 (more registers per row)
    const bool fp64_math = p->storage == LBM_F64 || p->storage == LBM_F32D || p->storage == LBM_F64T;
    if (p->tile_rows > 0)
        c->ty = p->tile_rows;
    else if (p->schedule == lbm::kScheduleTile)
        c->ty = (fp64_math || c->tile_waves == 8) ? 12 : 8;
    else if (p->schedule == lbm::kSchedulePipe)
        c->ty = 8;
    else
        c->ty = kDefaultMarchRows;
    c->nchunk = std::max(1, ny / c->ty);
    // workspace layout
    size_t o = 0;
    const size_t fbytes = align256((size_t)c->plane * 9 * storage_bytes(p->storage));
    const size_t nxy8 = align256((size_t)nx * ny * sizeof(double));
    c->off_f[0] = o; o += fbytes;
    c->off_f[1] = o; o += fbytes;
    c->off_rho = o; o += nxy8;
    c->off_vx = o; o += nxy8;
    c->off_vy = o; o += nxy8;
    c->off_ring = o; o += align256((size_t)kRingCap * lbm::kWallSlotVals * nx * sizeof(double));
    c->off_hist = o; o += align256((size_t)p->history_cap * sizeof(lbm_stress_summary));
    c->off_acc = o; o += 256;
    c->off_wscr = o; o += align256((size_t)kRingCap * 2 * lbm::kWallPartVals * sizeof(double));
    c->off_red = o; o += align256((size_t)lbm::kFieldReduceBlocks * 5 * sizeof(double));
    c->off_redout = o; o += 256;
    c->off_colmin = o; o += align256((size_t)nx * sizeof(double));
    c->off_centre = o; o += align256((size_t)nx * sizeof(double));
    c->off_tickets = o; o += (size_t)lbm::kTicketGroups * lbm::kTicketStride * sizeof(unsigned long long);
    c->off_sr = o; o += 256;
    c->total = o;
    c->check.rupture_step = -1;
    c->check.unstable_step = -1;
    *out = c;
    return LBM_OK;
}

lbm_status lbm_workspace(const lbm_ctx* c, size_t* bytes, size_t* align) {
    if (!c || !bytes) return LBM_EINVAL;
    *bytes = c->total;
    if (align) *align = 256;
    return LBM_OK;
}

lbm_status lbm_bind(lbm_ctx* c, void* device_ptr, size_t bytes, void* hip_stream) {
    if (!c) return LBM_EINVAL;
    if (!device_ptr || (reinterpret_cast<uintptr_t>(device_ptr) & 255))
        return fail(c, LBM_EINVAL, "workspace pointer must be non-null and 256-byte aligned");
    if (bytes < c->total) return fail(c, LBM_ENOMEM, "workspace of %zu bytes < %zu needed", bytes, c->total);
    const char* why = nullptr;
    if (lbm_status st = device_range_check(device_ptr, c->total, &why)) return fail(c, st, "workspace: %s", why);
    HIP_TRY(c, hipGetDevice(&c->device));
    HIP_TRY(c, lbm::noalloc_setup());  // this device's address of the static check scratch
    if (c->schedule == lbm::kSchedulePipe) {
        if (c->p.pipe_blocks > 0)
            c->pipe_blocks = c->p.pipe_blocks;
        else
            HIP_TRY(c, lbm::pipe_grid(c->p.storage, c->p.eos, c->ty, c->tile_waves, &c->pipe_blocks));
        if (c->pipe_blocks < lbm::kTicketGroups) c->pipe_blocks = lbm::kTicketGroups;
    }
    c->dev = static_cast<char*>(device_ptr);
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->bound = true;
    c->initialized = false;
    c->graphs.drop();
    c->adj.drop_graphs();
    return LBM_OK;
}

lbm_status lbm_state(const lbm_ctx* c, double* T, double* Tc, double* rho_g, double* rho_l, double* rho_w) {
    if (!c) return LBM_EINVAL;
    if (T) *T = c->eos.T;
    if (Tc) *Tc = c->eos.Tc;
    if (rho_g) *rho_g = c->rho_g;
    if (rho_l) *rho_l = c->rho_l;
    if (rho_w) *rho_w = c->rho_w;
    return LBM_OK;
}

lbm_status lbm_init_plug(lbm_ctx* c, double plug_len, double film, double x_center, double noise_amp,
                         uint64_t seed) {
    if (!c) return LBM_EINVAL;
    if (!(plug_len > 0) || plug_len > c->nx || !(film >= 0) || !(2 * film < c->ny) || !(noise_amp >= 0) ||
        std::isnan(c->rho_l) || (!std::isnan(x_center) && !std::isfinite(x_center)))
        return fail(c, LBM_EINVAL, "invalid plug: length %g film %g x_center %g noise %g (T/Tc %g)", plug_len, film,
                    x_center, noise_amp, c->p.T_over_Tc);
    if (!c->bound) return fail(c, LBM_ESTATE, "lbm_bind must come before initialisation");
    if (std::isnan(x_center)) x_center = c->nx / 4.0 + plug_len / 2.0;
    std::vector<double> rho;
    try {
        rho.resize((size_t)c->nx * c->ny);
    } catch (...) {
        return fail(c, LBM_ENOMEM, "host allocation of the initial density failed");
    }
    for (int y = 0; y < c->ny; ++y)
        for (int x = 0; x < c->nx; ++x) {
            const bool plug = x >= x_center - plug_len / 2.0 && x < x_center + plug_len / 2.0;
            const bool filmrow = y < film || y >= c->ny - film;
            const double base = (plug || filmrow) ? c->rho_l : c->rho_g;
            const uint64_t z = splitmix64_nth(seed, (uint64_t)y * c->nx + x);
            const double U = (double)(z >> 11) * 0x1.0p-53;
            rho[(size_t)y * c->nx + x] = base + noise_amp * (2.0 * U - 1.0);
        }
    HIP_TRY(c, hipMemcpyAsync(c->dev + c->off_rho, rho.data(), rho.size() * sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return init_from_device_rho(c);
}

lbm_status lbm_init_density(lbm_ctx* c, const double* rho) {
    if (!c || !rho) return LBM_EINVAL;
    for (long long i = 0, n = (long long)c->nx * c->ny; i < n; ++i)
        if (!(rho[i] > 0) || !std::isfinite(rho[i])) return fail(c, LBM_EINVAL, "density must be positive and finite");
    if (!c->bound) return fail(c, LBM_ESTATE, "lbm_bind must come before initialisation");
    HIP_TRY(c, hipMemcpyAsync(c->dev + c->off_rho, rho, (size_t)c->nx * c->ny * sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return init_from_device_rho(c);
}

namespace {

// One launch of the single-lattice step kernels: `nsteps` (1 or 2) steps from buffer `in`
// into the other one, wall arrays to ring slot `slot`.
hipError_t launch_k(const lbm_ctx* c, lbm::StepArgs& b, int in, int slot, int nsteps, bool emit, hipStream_t s) {
    b.fin = c->dev + c->off_f[in];
    b.fout = c->dev + c->off_f[1 - in];
    b.sr_par = in;
    set_wall_slot(b, c, slot);
    return nsteps == 2 ? lbm::launch_step2(b, c->p.storage, c->p.eos, emit, s)
                       : lbm::launch_step(b, c->p.storage, c->p.eos, emit, s);
}

lbm_status zero_tickets(lbm_ctx* c) {  // the pipelined schedule's counters start from zero per run of launches
    if (c->schedule == lbm::kSchedulePipe)
        HIP_TRY(c, lbm::launch_fill(c->at<double>(c->off_tickets), 0.0,
                                    (long long)lbm::kTicketGroups * lbm::kTicketStride, c->stream));
    return LBM_OK;
}

// Makes the field buffers hold the density and velocity of the latest step: when a call ended
// between checks they are older, and the latest step is launched again with field output from
// its input (the other distribution buffer).  The kernels are deterministic, so the run writes
// the same distributions, wall arrays and stochastic-rounding counter word as the first one.
lbm_status ensure_fields(lbm_ctx* c) {
    if (c->fields_step == c->steps) return LBM_OK;
    if (!c->prev_valid || c->last_slot < 0)
        return fail(c, LBM_ESTATE, "the fields of step %lld cannot be formed: the previous state was replaced",
                    (long long)c->steps);
    lbm::StepArgs a = make_args(c);
    lbm_status s = zero_tickets(c);
    if (s) return s;
    a.launch = 0;
    HIP_TRY(c, launch_k(c, a, 1 - c->cur, c->last_slot, 1, true, c->stream));
    c->fields_step = c->steps;
    return LBM_OK;
}

// A check at the current step (forming its fields first), unless one already ran there.
lbm_status check_now(lbm_ctx* c) {
    if (c->check.step == c->steps) return LBM_OK;
    lbm_status s = ensure_fields(c);
    if (s) return s;
    return run_check(c);
}

// n steps, or (dry) only the capture of the graphs those steps would replay, with
// nothing launched and the context left as it was.
//
// Checks run at every multiple of check_every: the step there emits the fields, the wall ring
// is reduced and the check's results are read back (one host synchronisation).  Between checks
// the steps are replayed from captured graphs of graph_steps launches and one graph for the
// rest of the run.  A call ends with the reduction of its steps' wall ring queued on the stream
// and returns without waiting for the device.
lbm_status step_impl(lbm_ctx* c, int64_t n, bool dry) {
    struct Cursor {
        int cur, ring_fill, last_slot;
        int64_t steps, ring_first_step;
    };
    const Cursor saved{c->cur, c->ring_fill, c->last_slot, c->steps, c->ring_first_step};
    lbm::StepArgs a = make_args(c);
    if (!dry && n > 0) {
        lbm_status s = zero_tickets(c);
        if (s) return s;
    }
    a.launch = 0;
    const int G = c->graph_steps();
    const int L = c->steps_per_launch();  // steps per launch (1 or 2); G is a multiple of it
    auto flush = [&]() -> lbm_status {
        if (!dry) return flush_wall(c);
        c->ring_first_step += c->ring_fill;
        c->ring_fill = 0;
        return LBM_OK;
    };
    const bool walls = !c->p.y_periodic;
    auto advance = [&](int m, int launches) {
        if (launches & 1) c->cur = 1 - c->cur;
        c->last_slot = c->ring_fill + m - 1;
        c->ring_fill += m;
        c->steps += m;
    };
    // m steps launched kernel by kernel (L steps per launch while more than one step remains)
    auto eager = [&](int64_t m, bool emit_last) -> lbm_status {
        for (int64_t k = 0; k < m;) {
            const int mm = (L == 2 && m - k >= 2) ? 2 : 1;
            if (c->ring_fill + mm > kRingCap) {
                lbm_status s = flush();
                if (s) return s;
            }
            const bool emit = emit_last && k + mm == m;
            if (!dry) HIP_TRY(c, launch_k(c, a, c->cur, c->ring_fill, mm, emit, c->stream));
            a.launch += 1;
            advance(mm, 1);
            k += mm;
        }
        return LBM_OK;
    };
    int64_t done = 0;
    lbm_status result = LBM_OK;
    while (done < n) {
        const int64_t next_check = (c->steps / c->p.check_every + 1) * c->p.check_every;
        const int64_t seg = std::min<int64_t>(n - done, next_check - c->steps);
        const bool check = c->steps + seg == next_check;
        // the step that emits for a check, and with two steps per launch the last step of
        // the call, are one-step launches
        const int64_t tail = (check || L == 2) ? 1 : 0;
        int64_t body = seg - tail;
        while (body > 0) {
            int m = G > 0 ? (int)std::min<int64_t>(body, G) : 0;
            if (L == 2) m &= ~1;
            hipGraphExec_t* ge = nullptr;
            // the call's last run (no check, no one-step launch after it) ends with the flush
            const bool with_flush = walls && !check && tail == 0 && m == body;
            if (m > 0) {
                if (c->ring_fill + m > kRingCap) {
                    lbm_status s = flush();
                    if (s) return s;
                }
                ge = c->graphs.entry(c->cur, c->ring_fill, m, G, with_flush);
            }
            if (!ge) {  // no graphs, or the cache of short runs is full
                lbm_status s = eager(m > 0 ? m : body, false);
                if (s) return s;
                body -= m > 0 ? m : body;
                continue;
            }
            const int nl = m / L;  // launches in the graph; each flips the buffers once
            if (!*ge) {
                const int par = c->cur, fill0 = c->ring_fill;
                auto launch = [&](int j, hipStream_t s) {
                    if (j == nl)  // the flush of every ring slot written so far
                        return lbm::launch_wall_reduce(c->at<double>(c->off_ring), fill0 + m, c->nx,
                                                       c->at<lbm_stress_summary>(c->off_hist), c->p.history_cap,
                                                       c->at<double>(c->off_wscr), c->at<double>(c->off_acc), s);
                    lbm::StepArgs b = a;
                    return launch_k(c, b, (par + j) & 1, fill0 + L * j, L, false, s);
                };
                HIP_TRY(c, capture_graph(c->graphs, nl + (with_flush ? 1 : 0), launch, ge));
            }
            if (!dry) HIP_TRY(c, hipGraphLaunch(*ge, c->stream));
            advance(m, nl);
            body -= m;
            if (with_flush) {  // flushed inside the graph
                c->ring_first_step += c->ring_fill;
                c->ring_fill = 0;
            }
        }
        if (tail) {
            lbm_status s = eager(1, check);
            if (s) return s;
        }
        done += seg;
        if (!dry) {
            c->prev_valid = true;
            if (check) c->fields_step = c->steps;
        }
        if (!check) break;  // the end of the call, between checks
        lbm_status s = flush();
        if (s) return s;
        if (!dry) {
            s = run_check(c);
            if (s) return s;
        }
    }
    if (dry) {
        c->cur = saved.cur;
        c->ring_fill = saved.ring_fill;
        c->last_slot = saved.last_slot;
        c->steps = saved.steps;
        c->ring_first_step = saved.ring_first_step;
        return LBM_OK;
    }
    lbm_status s = flush();  // queued: every step's wall summaries without waiting for them
    if (s) return s;
    if (result == LBM_OK && c->check.unstable_step >= 0)
        return fail(c, LBM_EUNSTABLE, "state is unstable since step %lld", (long long)c->check.unstable_step);
    return result;
}

}  // namespace

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
    if (!c || n < 0) return LBM_EINVAL;
    if (c->in_batch) return fail(c, LBM_ESTATE, "this context belongs to a batch: step it with lbm_batch_step");
    if (!c->bound || !c->initialized) return fail(c, LBM_ESTATE, "lbm_step needs lbm_bind and an initialisation");
    return step_impl(c, n, false);
}

lbm_status lbm_capture(lbm_ctx* c, int64_t n) {
    if (!c || n < 0) return LBM_EINVAL;
    if (c->in_batch) return fail(c, LBM_ESTATE, "this context belongs to a batch: use lbm_batch_capture");
    if (!c->bound || !c->initialized) return fail(c, LBM_ESTATE, "lbm_capture needs lbm_bind and an initialisation");
    return step_impl(c, n, true);
}

lbm_status lbm_step_count(const lbm_ctx* c, int64_t* steps) {
    if (!c || !steps) return LBM_EINVAL;
    *steps = c->steps;
    return LBM_OK;
}

lbm_status lbm_fields(lbm_ctx* c, double* rho, double* vx, double* vy) {
    if (!c) return LBM_EINVAL;
    if (!c->initialized) return fail(c, LBM_ESTATE, "not initialised");
    if (lbm_status st = ensure_fields(c)) return st;
    const size_t bytes = (size_t)c->nx * c->ny * sizeof(double);
    if (rho) HIP_TRY(c, hipMemcpyAsync(rho, c->dev + c->off_rho, bytes, hipMemcpyDeviceToHost, c->stream));
    if (vx) HIP_TRY(c, hipMemcpyAsync(vx, c->dev + c->off_vx, bytes, hipMemcpyDeviceToHost, c->stream));
    if (vy) HIP_TRY(c, hipMemcpyAsync(vy, c->dev + c->off_vy, bytes, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_wall_stress(lbm_ctx* c, double* tau_bot, double* tau_top, double* p_bot, double* p_top,
                           lbm_stress_summary* s) {
    if (!c) return LBM_EINVAL;
    if (!c->initialized) return fail(c, LBM_ESTATE, "not initialised");
    const size_t nxb = (size_t)c->nx * sizeof(double);
    double* outs[4] = {tau_bot, tau_top, p_bot, p_top};
    for (int q = 0; q < 4; ++q) {
        if (!outs[q]) continue;
        if (c->last_slot < 0 || c->p.y_periodic) {  // no step yet, or no walls: zeros
            std::memset(outs[q], 0, nxb);
            continue;
        }
        const char* src = c->dev + c->off_ring + ((size_t)c->last_slot * lbm::kWallSlotVals + q) * nxb;
        HIP_TRY(c, hipMemcpyAsync(outs[q], src, nxb, hipMemcpyDeviceToHost, c->stream));
    }
    if (s) {
        std::memset(s, 0, sizeof *s);
        if (c->steps >= c->hist_first && !c->p.y_periodic) {
            const size_t idx = (size_t)((c->steps - 1) % c->p.history_cap);
            HIP_TRY(c, hipMemcpyAsync(s, c->dev + c->off_hist + idx * sizeof(lbm_stress_summary),
                                      sizeof(lbm_stress_summary), hipMemcpyDeviceToHost, c->stream));
        }
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_stress_history(lbm_ctx* c, lbm_stress_summary* buf, int64_t cap, int64_t* n_out) {
    if (!c || !n_out || cap < 0 || (cap > 0 && !buf)) return LBM_EINVAL;
    if (!c->initialized) return fail(c, LBM_ESTATE, "not initialised");
    const int64_t have = c->p.y_periodic ? 0 : std::min<int64_t>(c->steps - c->hist_first + 1, c->p.history_cap);
    const int64_t n = std::min(have, cap);
    std::vector<lbm_stress_summary> ring(c->p.history_cap);
    if (n > 0) {
        HIP_TRY(c, hipMemcpyAsync(ring.data(), c->dev + c->off_hist, ring.size() * sizeof(lbm_stress_summary),
                                  hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        for (int64_t k = 0; k < n; ++k) {
            const int64_t step = c->steps - n + 1 + k;
            buf[k] = ring[(size_t)((step - 1) % c->p.history_cap)];
        }
    }
    *n_out = n;
    return LBM_OK;
}

lbm_status lbm_check_state(lbm_ctx* c, lbm_check_result* out) {
    if (!c || !out) return LBM_EINVAL;
    if (c->initialized && c->bound) {
        lbm_status s = check_now(c);
        if (s != LBM_OK && s != LBM_EUNSTABLE) return s;  // instability is reported in the result
    }
    *out = c->check;
    return LBM_OK;
}

lbm_status lbm_check_state_noalloc(lbm_ctx* c, lbm_check_result* out) {
    if (!c || !out) return LBM_EINVAL;
    if (!c->bound || !c->initialized)
        return fail(c, LBM_ESTATE, "lbm_check_state_noalloc needs a bound, initialised lattice");
    if (c->nx > lbm::kNoAllocMaxNx)
        return fail(c, LBM_EINVAL, "lbm_check_state_noalloc: nx = %d exceeds the %d columns its static scratch holds",
                    c->nx, lbm::kNoAllocMaxNx);
    if (c->check.step != c->steps) {
        lbm_status s = ensure_fields(c);
        if (s) return s;
        const double mid = 0.5 * (c->rho_g + c->rho_l);
        const bool two_phase = std::isfinite(mid);
        double h[9];
        HIP_TRY(c, lbm::noalloc_check(c->device, c->at<double>(c->off_rho), c->at<double>(c->off_vx),
                                      c->at<double>(c->off_vy), c->nx, c->ny, two_phase ? mid : 0.0, h, c->stream));
        s = check_apply(c, h, two_phase ? h[6] : NAN, two_phase ? h[7] : NAN, two_phase ? (int)h[5] : 0);
        if (s != LBM_OK && s != LBM_EUNSTABLE) return s;  // instability is reported in the result
    }
    *out = c->check;
    return LBM_OK;
}

// Same shift arithmetic as the device codecs: one fused multiply-add with 9 w_i and the shift unit q.
static float host_k(int i) { return i == 0 ? 4.0f : (i < 5 ? 1.0f : 0.25f); }

lbm_status lbm_get_f(lbm_ctx* c, double* f) {
    if (!c || !f) return LBM_EINVAL;
    if (!c->initialized) return fail(c, LBM_ESTATE, "not initialised");
    const size_t sb = storage_bytes(c->p.storage);
    std::vector<unsigned char> raw((size_t)c->plane * 9 * sb);
    HIP_TRY(c, hipMemcpyAsync(raw.data(), c->dev + c->off_f[c->cur], raw.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const float r0 = (float)c->shift_q;
    for (int i = 0; i < 9; ++i)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                const size_t src = (size_t)i * c->plane + (size_t)y * c->pitch + x;
                double v;
                switch (c->p.storage) {
                    case LBM_F64: std::memcpy(&v, raw.data() + src * 8, 8); break;
                    case LBM_F64T: std::memcpy(&v, raw.data() + src * 16, 8); break;
                    case LBM_F32:
                    case LBM_F32D: { float t; std::memcpy(&t, raw.data() + src * 4, 4); v = t; break; }
                    case LBM_F32S: { float t; std::memcpy(&t, raw.data() + src * 4, 4); v = (double)std::fmaf(host_k(i), r0, t); break; }
                    case LBM_F16S:
                    case LBM_F16R: {
                        _Float16 h;
                        std::memcpy(&h, raw.data() + src * 2, 2);
                        v = (double)std::fmaf(host_k(i), r0, (float)h);
                        break;
                    }
                    default: {
                        uint16_t h;
                        std::memcpy(&h, raw.data() + src * 2, 2);
                        uint32_t u = (uint32_t)h << 16;
                        float t;
                        std::memcpy(&t, &u, 4);
                        v = (double)std::fmaf(host_k(i), r0, t);
                    }
                }
                f[((size_t)i * c->ny + y) * c->nx + x] = v;
            }
    return LBM_OK;
}

lbm_status lbm_set_f(lbm_ctx* c, const double* f) {
    if (!c || !f) return LBM_EINVAL;
    if (!c->bound) return fail(c, LBM_ESTATE, "lbm_bind must come first");
    if (c->initialized) {  // the fields stay those of the latest step
        lbm_status s = ensure_fields(c);
        if (s) return s;
    }
    const size_t sb = storage_bytes(c->p.storage);
    std::vector<unsigned char> raw((size_t)c->plane * 9 * sb, 0);
    const float r0 = (float)c->shift_q;
    for (int i = 0; i < 9; ++i)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                const size_t dst = (size_t)i * c->plane + (size_t)y * c->pitch + x;
                const double v = f[((size_t)i * c->ny + y) * c->nx + x];
                switch (c->p.storage) {
                    case LBM_F64: std::memcpy(raw.data() + dst * 8, &v, 8); break;
                    case LBM_F64T: std::memcpy(raw.data() + dst * 16, &v, 8); break;  // tangent zero
                    case LBM_F32:
                    case LBM_F32D: { const float t = (float)v; std::memcpy(raw.data() + dst * 4, &t, 4); break; }
                    case LBM_F32S: { const float t = std::fmaf(-host_k(i), r0, (float)v); std::memcpy(raw.data() + dst * 4, &t, 4); break; }
                    case LBM_F16S:
                    case LBM_F16R: {
                        const _Float16 h = (_Float16)std::fmaf(-host_k(i), r0, (float)v);
                        std::memcpy(raw.data() + dst * 2, &h, 2);
                        break;
                    }
                    default: {
                        const float t = std::fmaf(-host_k(i), r0, (float)v);
                        uint32_t u;
                        std::memcpy(&u, &t, 4);
                        u += 0x7FFFu + ((u >> 16) & 1u);
                        const uint16_t h = (uint16_t)(u >> 16);
                        std::memcpy(raw.data() + dst * 2, &h, 2);
                    }
                }
            }
    HIP_TRY(c, hipMemcpyAsync(c->dev + c->off_f[c->cur], raw.data(), raw.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (!c->initialized) {
        lbm_status s = reset_diagnostics(c);
        if (s) return s;
        c->initialized = true;
    }
    c->prev_valid = false;  // the latest step's input no longer leads to the state
    return LBM_OK;
}

lbm_status lbm_reset_stress_extremes(lbm_ctx* c) {
    if (!c) return LBM_EINVAL;
    if (!c->initialized) return fail(c, LBM_ESTATE, "not initialised");
    double* acc = c->at<double>(c->off_acc);
    for (int q = 0; q < 4; ++q)  // every lbm_step call flushes the wall ring, so no earlier step is pending
        HIP_TRY(c, lbm::launch_fill(acc + 2 + 2 * q, (q % 2 == 0) ? -INFINITY : INFINITY, 2, c->stream));
    return LBM_OK;
}

lbm_status lbm_set_tangent(lbm_ctx* c, const double* dtheta) {
    if (!c || !dtheta) return LBM_EINVAL;
    if (c->p.storage != LBM_F64T) return fail(c, LBM_EINVAL, "lbm_set_tangent needs F64T storage");
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(dtheta[k])) return fail(c, LBM_EINVAL, "tangent direction must be finite");
    if (c->p.eos == LBM_EOS_PR && (dtheta[1] != 0.0 || dtheta[2] != 0.0))
        return fail(c, LBM_EINVAL, "PR tangents support d dp and d T only");
    if (c->initialized && c->bound) {  // a rerun of the latest step with other tangents would change the state
        lbm_status s = ensure_fields(c);
        if (s) return s;
        c->prev_valid = false;
    }
    for (int k = 0; k < 4; ++k) c->dtheta[k] = dtheta[k];
    c->graphs.drop();  // the step coefficients' tangents are kernel arguments
    return LBM_OK;
}

lbm_status lbm_get_f_tangent(lbm_ctx* c, double* df) {
    if (!c || !df) return LBM_EINVAL;
    if (c->p.storage != LBM_F64T) return fail(c, LBM_EINVAL, "lbm_get_f_tangent needs F64T storage");
    if (!c->initialized) return fail(c, LBM_ESTATE, "not initialised");
    std::vector<unsigned char> raw((size_t)c->plane * 9 * 16);
    HIP_TRY(c, hipMemcpyAsync(raw.data(), c->dev + c->off_f[c->cur], raw.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < 9; ++i)
        for (int y = 0; y < c->ny; ++y)
            for (int x = 0; x < c->nx; ++x) {
                const size_t src = (size_t)i * c->plane + (size_t)y * c->pitch + x;
                std::memcpy(&df[((size_t)i * c->ny + y) * c->nx + x], raw.data() + src * 16 + 8, 8);
            }
    return LBM_OK;
}

// ---- tile autotuner ----------------------------------------------------------------

}  // extern "C"

namespace {

struct TileShape {
    int rows, waves;
};
// Tile shapes of the tile schedule (schedule_ok), in the order they are tried.
constexpr TileShape kTileShapes[] = {{8, 4}, {12, 4}, {20, 4}, {28, 4}, {12, 8}, {20, 8}, {28, 8}};

// Step arguments for timing trials: the wall arrays go to a slot of the (flushed)
// wall ring other than the latest step's, so a trial leaves every diagnostic
// the caller can read untouched.
lbm::StepArgs trial_args(const lbm_ctx* c) {
    lbm::StepArgs a = make_args(c);
    set_wall_slot(a, c, (c->last_slot + 1) % kRingCap);
    a.fin = c->dev + c->off_f[c->cur];  // every trial reads the current state and writes the other buffer
    a.fout = c->dev + c->off_f[1 - c->cur];
    return a;
}

// Mean time per launch of `trials` launches after one warm-up launch.
template <class F>
hipError_t time_launches(hipStream_t s, int trials, F&& launch, double* us) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int k = 0; k < trials && e == hipSuccess; ++k) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    *us = 1e3 * ms / trials;
    return e;
}

}  // namespace

extern "C" {

lbm_status lbm_launch_config(const lbm_ctx* c, int* tile_rows, int* tile_waves, int* fused_steps, int* graph_steps) {
    if (!c) return LBM_EINVAL;
    if (tile_rows) *tile_rows = c->ty;
    if (tile_waves) *tile_waves = c->tile_waves;
    if (fused_steps) *fused_steps = c->steps_per_launch();
    if (graph_steps) *graph_steps = c->graph_steps();
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx* c, int trial_steps, int* tile_rows, int* tile_waves, double* us_per_step) {
    if (!c || trial_steps < 1) return LBM_EINVAL;
    if (c->in_batch) return fail(c, LBM_ESTATE, "a batch case is tuned with lbm_batch_autotune");
    if (!c->bound || !c->initialized) return fail(c, LBM_ESTATE, "lbm_autotune needs an initialised lattice");
    if (c->schedule != lbm::kScheduleTile || c->p.storage == LBM_F64T)
        return fail(c, LBM_EINVAL, "lbm_autotune tunes the tile schedule (not F64T storage)");
    lbm_status s = flush_wall(c);
    if (s) return s;
    s = ensure_fields(c);  // the trials overwrite the latest step's input
    if (s) return s;
    c->prev_valid = false;
    double best = INFINITY;
    TileShape pick = {c->ty, c->tile_waves};
    for (const TileShape& t : kTileShapes) {
        lbm::StepArgs a = trial_args(c);
        a.ty = t.rows;
        a.tile_waves = t.waves;
        double us = 0;
        HIP_TRY(c, time_launches(c->stream, trial_steps,
                                 [&] { return lbm::launch_step(a, c->p.storage, c->p.eos, false, c->stream); }, &us));
        if (us < best) { best = us; pick = t; }
    }
    // two steps per launch, where the storage has the two-step kernel; their two wall
    // arrays go to two consecutive ring slots, neither of them the latest step's
    int fused = 1;
    if (c->p.storage != LBM_F16R) {
        lbm::StepArgs a = trial_args(c);
        set_wall_slot(a, c, c->last_slot + 1 <= kRingCap - 2 ? c->last_slot + 1 : 0);
        double us = 0;
        HIP_TRY(c, time_launches(c->stream, (trial_steps + 1) / 2,
                                 [&] { return lbm::launch_step2(a, c->p.storage, c->p.eos, false, c->stream); }, &us));
        if (0.5 * us < best) {
            best = 0.5 * us;
            fused = 2;
        }
    }
    c->ty = c->p.tile_rows = pick.rows;
    c->tile_waves = c->p.tile_waves = pick.waves;
    c->p.fused_steps = fused;
    c->nchunk = std::max(1, c->ny / c->ty);
    c->graphs.drop();  // the launch configuration is part of the captured launches
    if (tile_rows) *tile_rows = pick.rows;
    if (tile_waves) *tile_waves = pick.waves;
    if (us_per_step) *us_per_step = best;
    return LBM_OK;
}

// ---- reverse-mode sensitivities ------------------------------------------------

namespace {
constexpr int kAdjRing = 64;  // adjoint launches whose parameter partials are reduced together

size_t adjoint_arith_bytes(int storage) { return storage == LBM_F32 ? 4 : 8; }

// Adjoint tile: output rows and waves per block.  Measured on the 1024x256 and
// 4096x512 channels (FP32 and FP64): 4-row tiles (one row per wave, the most
// blocks) are fastest below 1M nodes, 12-row tiles (less halo) above.
void adjoint_tile_shape(const lbm_ctx* c, int* ty, int* waves) {
    *ty = (long long)c->nx * c->ny >= (1LL << 20) ? 12 : 4;
    *waves = 8;
}

lbm_status adjoint_layout(const lbm_ctx* c, int64_t nsteps, int64_t segment, lbm_ctx::Adjoint& A) {
    if (c->p.storage != LBM_F64 && c->p.storage != LBM_F32 && c->p.storage != LBM_F32D) return LBM_EINVAL;
    if (c->schedule != lbm::kScheduleTile || nsteps < 1 || segment < 0 || segment > nsteps) return LBM_EINVAL;
    A.n = nsteps;
    A.seg = segment > 0 ? segment : (int64_t)std::ceil(std::sqrt((double)nsteps));
    A.nckpt = (nsteps + A.seg - 1) / A.seg;
    const size_t ab = adjoint_arith_bytes(c->p.storage);
    A.state = align256((size_t)c->plane * 9 * storage_bytes(c->p.storage));
    // adjoint fields are addressed with 32-bit byte offsets like the distributions
    if ((unsigned long long)c->plane * 9 * ab >= (1ULL << 32)) return LBM_EINVAL;
    A.lam = align256((size_t)c->plane * 9 * ab);
    A.fld = align256((size_t)lbm::adjoint_field_elems(c->plane, c->nx) * ab);
    adjoint_tile_shape(c, &A.ty, &A.waves);
    A.blocks = lbm::adjoint_blocks(c->nx, c->ny, A.ty);
    size_t o = 0;
    A.off_ckpt = o; o += (size_t)A.nckpt * A.state;
    A.off_pp = o; o += 2 * A.state;               // the recompute's two states
    A.off_fld = o; o += 2 * (size_t)A.seg * A.fld;  // forward fields of each step of two segments
    A.off_lam[0] = o; o += A.lam;
    A.off_lam[1] = o; o += A.lam;
    A.off_tw = o; o += align256(2 * (size_t)A.seg * 2 * c->nx * sizeof(double));  // their wall shears
    A.off_seed = o; o += align256(2 * (size_t)A.seg * 2 * c->nx * sizeof(double));  // and peak-objective seeds
    A.ring_cap = (int)std::max<int64_t>(A.seg, kAdjRing);  // adjoint launches between reductions
    A.off_part = o; o += align256((size_t)A.ring_cap * A.blocks * 4 * sizeof(double));
    A.off_red = o; o += align256((size_t)A.ring_cap * 4 * sizeof(double));
    A.off_acc = o; o += 256;
    A.off_pw = o; o += align256((size_t)4 * c->nx * sizeof(double));
    A.off_g0 = o; o += align256((size_t)9 * c->nx * c->ny * sizeof(double));
    A.total = o;
    return LBM_OK;
}
}  // namespace

lbm_status lbm_adjoint_workspace(const lbm_ctx* c, int64_t nsteps, int64_t segment, size_t* bytes) {
    if (!c || !bytes) return LBM_EINVAL;
    lbm_ctx::Adjoint A;
    lbm_status s = adjoint_layout(c, nsteps, segment, A);
    if (s) return s;
    *bytes = A.total;
    return LBM_OK;
}

lbm_status lbm_adjoint_bind(lbm_ctx* c, void* device_ptr, size_t bytes, int64_t nsteps, int64_t segment) {
    if (!c) return LBM_EINVAL;
    if (c->in_batch) return fail(c, LBM_ESTATE, "a batch case has no adjoint");
    lbm_ctx::Adjoint A;
    if (adjoint_layout(c, nsteps, segment, A))
        return fail(c, LBM_EINVAL, "adjoint: storage must be f64, f32 or f32d with the tile schedule, "
                                   "1 <= nsteps and 0 <= segment <= nsteps");
    if (!device_ptr || (reinterpret_cast<uintptr_t>(device_ptr) & 255))
        return fail(c, LBM_EINVAL, "adjoint workspace pointer must be non-null and 256-byte aligned");
    if (bytes < A.total) return fail(c, LBM_ENOMEM, "adjoint workspace of %zu bytes < %zu needed", bytes, A.total);
    const char* why = nullptr;
    if (lbm_status st = device_range_check(device_ptr, A.total, &why))
        return fail(c, st, "adjoint workspace: %s", why);
    A.dev = static_cast<char*>(device_ptr);
    A.bound = true;
    c->adj = A;
    return LBM_OK;
}

lbm_status lbm_adjoint_objective(lbm_ctx* c, int objective) {
    if (!c || (objective != LBM_J_SUM_TAU2 && objective != LBM_J_PEAK_TAU2)) return LBM_EINVAL;
    if (!c->adj.bound) return fail(c, LBM_ESTATE, "lbm_adjoint_bind must come first");
    if (c->adj.objective != objective) {
        c->adj.objective = objective;
        c->adj.recorded = c->adj.swept = false;  // J of the record was the other objective
        c->adj.drop_graphs();                    // the recompute graphs include the seeds or not
    }
    return LBM_OK;
}

lbm_status lbm_adjoint_forward(lbm_ctx* c, double* J) {
    if (!c) return LBM_EINVAL;
    if (!c->adj.bound) return fail(c, LBM_ESTATE, "lbm_adjoint_bind must come first");
    if (!c->bound || !c->initialized) return fail(c, LBM_ESTATE, "lbm_adjoint_forward needs an initialised lattice");
    lbm_ctx::Adjoint& A = c->adj;
    A.recorded = A.swept = false;
    lbm_status s = flush_wall(c);
    if (s) return s;
    double acc0[2], acc1[2];
    HIP_TRY(c, hipMemcpyAsync(acc0, c->dev + c->off_acc, sizeof acc0, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const size_t fbytes = (size_t)c->plane * 9 * storage_bytes(c->p.storage);
    for (int64_t k = 0; k < A.nckpt; ++k) {
        HIP_TRY(c, hipMemcpyAsync(A.dev + A.off_ckpt + (size_t)k * A.state, c->dev + c->off_f[c->cur], fbytes,
                                  hipMemcpyDeviceToDevice, c->stream));
        s = step_impl(c, std::min(A.seg, A.n - k * A.seg), false);  // checks at their cadence only
        if (s) return s;
    }
    s = check_now(c);  // a record that went unstable is not kept
    if (s) return s;
    HIP_TRY(c, hipMemcpyAsync(acc1, c->dev + c->off_acc, sizeof acc1, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int q = A.objective == LBM_J_PEAK_TAU2 ? 0 : 1;  // acc: [0] int peak tau^2, [1] int sum tau^2
    A.J = acc1[q] - acc0[q];  // the objective over the recorded steps
    A.recorded = true;
    if (J) *J = A.J;
    return LBM_OK;
}

lbm_status lbm_adjoint_backward(lbm_ctx* c, double seed, double* grad) {
    if (!c || !grad || !std::isfinite(seed)) return LBM_EINVAL;
    lbm_ctx::Adjoint& A = c->adj;
    if (!A.bound || !A.recorded) return fail(c, LBM_ESTATE, "lbm_adjoint_backward needs lbm_adjoint_forward first");
    const int storage = c->p.storage, eos = c->p.eos;
    lbm::StepArgs base = make_args(c);
    double* tw = reinterpret_cast<double*>(A.dev + A.off_tw);
    double* part = reinterpret_cast<double*>(A.dev + A.off_part);
    double* acc = reinterpret_cast<double*>(A.dev + A.off_acc);
    double* red = reinterpret_cast<double*>(A.dev + A.off_red);
    auto pp = [&](int64_t i) { return A.dev + A.off_pp + (size_t)(i & 1) * A.state; };
    // step i of the segment held in field buffer b: its forward fields and wall shears
    auto fld = [&](int b, int64_t i) { return A.dev + A.off_fld + ((size_t)b * A.seg + (size_t)i) * A.fld; };
    auto twp = [&](int b, int64_t i) { return tw + ((size_t)b * A.seg + (size_t)i) * 2 * c->nx; };
    double* seeds = reinterpret_cast<double*>(A.dev + A.off_seed);
    auto seedp = [&](int b, int64_t i) { return seeds + ((size_t)b * A.seg + (size_t)i) * 2 * c->nx; };
    const bool peak = A.objective == LBM_J_PEAK_TAU2;
    HIP_TRY(c, lbm::launch_fill(reinterpret_cast<double*>(A.dev + A.off_lam[0]), 0.0, (long long)(A.lam / 8), c->stream));
    HIP_TRY(c, lbm::launch_fill(acc, 0.0, 4, c->stream));
    A.cur = 0;
    lbm::StepArgs fa = base;  // forward recompute: wall shear to the per-step slots, other diagnostics to scratch
    fa.p_w = reinterpret_cast<double*>(A.dev + A.off_pw);
    fa.dtau_w = fa.p_w + 2 * (size_t)c->nx;
    lbm::AdjArgs aa{};
    aa.s = base;
    aa.nstrip = (c->nx + lbm::kAdjStripOut - 1) / lbm::kAdjStripOut;
    aa.ty = A.ty;
    aa.waves = A.waves;
    const bool graphs = c->graph_steps() > 0;
    if (!A.aux) HIP_TRY(c, hipStreamCreateWithFlags(&A.aux, hipStreamNonBlocking));
    // Below 1M nodes neither kernel fills the chip and the overlap pays (1024x256 FP32: backward sweep 0.456 ->
    // 0.329 s); on 4096x512 both stream close to the roofline and contend (0.177 -> 0.182 s), so there the
    // recompute runs on the main stream, in the same order.
    const hipStream_t rs = (long long)c->nx * c->ny < (1LL << 20) ? A.aux : c->stream;
    for (hipEvent_t* e : {&A.ev_start, &A.ev_rec[0], &A.ev_rec[1], &A.ev_adj[0], &A.ev_adj[1]})
        if (!*e) HIP_TRY(c, hipEventCreateWithFlags(e, hipEventDisableTiming));
    // Recompute launch j of a segment into field buffer b: step start + 1 + j from pp(j) to pp(j + 1).
    auto rec_launch = [&](int b, int64_t j, hipStream_t s) -> hipError_t {
        if (j == A.seg) return lbm::launch_peak_seed(twp(b, 0), seedp(b, 0), c->nx, (int)A.seg, s);  // graphs only
        lbm::StepArgs r = fa;
        r.fin = pp(j);
        r.fout = pp(j + 1);
        r.save = fld(b, j);
        r.tau_w = twp(b, j);
        return lbm::launch_step_save(r, storage, eos, s);
    };
    // Adjoint launch m (m < len) of a segment in buffer b, from its last step down; launch len: the reduction.
    auto adj_launch = [&](int b, int64_t len, int cur0, int ring0, int64_t m, hipStream_t s) -> hipError_t {
        if (m == len) return lbm::launch_adjoint_reduce(part, (int)(ring0 + len), A.blocks, red, acc, s);
        const int64_t i = len - 1 - m;
        const int par = (cur0 + (int)m) & 1;
        lbm::AdjArgs r = aa;
        r.fld = fld(b, i);
        r.lam_in = A.dev + A.off_lam[par];
        r.lam_out = A.dev + A.off_lam[1 - par];
        r.tau_w = twp(b, i);
        r.seed = peak ? seedp(b, i) : nullptr;
        r.partial = part + (size_t)(ring0 + m) * A.blocks * 4;
        return lbm::launch_adjoint(r, storage, eos, s);
    };
    auto seg_len = [&](int64_t k) { return std::min(A.seg, A.n - k * A.seg); };
    // Segment k's recompute on stream rs, into buffer k & 1, from a copy of its checkpoint.
    auto recompute = [&](int64_t k) -> lbm_status {
        const int b = (int)(k & 1);
        const int64_t len = seg_len(k);
        HIP_TRY(c, hipMemcpyAsync(pp(0), A.dev + A.off_ckpt + (size_t)k * A.state, A.state, hipMemcpyDeviceToDevice,
                                  rs));
        if (len == A.seg && graphs) {
            if (!A.rec_graph[b]) {  // the recompute, then (peak objective) the seeds of its steps
                auto launch = [&](int j, hipStream_t s) { return rec_launch(b, j, s); };
                HIP_TRY(c, capture_graph(c->graphs, (int)len + (peak ? 1 : 0), launch, &A.rec_graph[b]));
            }
            HIP_TRY(c, hipGraphLaunch(A.rec_graph[b], rs));
        } else {
            for (int64_t j = 0; j < len; ++j) HIP_TRY(c, rec_launch(b, j, rs));
            if (peak) HIP_TRY(c, lbm::launch_peak_seed(twp(b, 0), seedp(b, 0), c->nx, (int)len, rs));
        }
        HIP_TRY(c, hipEventRecord(A.ev_rec[b], rs));
        return LBM_OK;
    };
    // The recompute stream starts after everything queued so far (the record, the fills).
    HIP_TRY(c, hipEventRecord(A.ev_start, c->stream));
    HIP_TRY(c, hipStreamWaitEvent(rs, A.ev_start, 0));
    lbm_status st = recompute(A.nckpt - 1);
    if (st) return st;
    int ring = 0;
    for (int64_t k = A.nckpt - 1; k >= 0; --k) {
        const int b = (int)(k & 1);
        const int64_t len = seg_len(k);
        if (k >= 1) {
            // segment k - 1 goes to the buffer segment k + 1's sweep read: wait for that sweep
            if (k + 1 <= A.nckpt - 1) HIP_TRY(c, hipStreamWaitEvent(rs, A.ev_adj[(k + 1) & 1], 0));
            st = recompute(k - 1);
            if (st) return st;
        }
        HIP_TRY(c, hipStreamWaitEvent(c->stream, A.ev_rec[b], 0));
        if (len == A.seg && graphs) {
            // a full segment: the captured sweep (its reduction included)
            if (ring > 0) {
                HIP_TRY(c, lbm::launch_adjoint_reduce(part, ring, A.blocks, red, acc, c->stream));
                ring = 0;
            }
            hipGraphExec_t& ge = A.adj_graph[b][A.cur];
            if (!ge) {
                const int cur0 = A.cur;
                auto launch = [&](int m, hipStream_t s) { return adj_launch(b, len, cur0, 0, m, s); };
                HIP_TRY(c, capture_graph(c->graphs, (int)(len + 1), launch, &ge));
            }
            HIP_TRY(c, hipGraphLaunch(ge, c->stream));
        } else {
            // the last (shorter) segment, or every segment without graphs: direct launches
            if (ring + len > A.ring_cap) {
                HIP_TRY(c, lbm::launch_adjoint_reduce(part, ring, A.blocks, red, acc, c->stream));
                ring = 0;
            }
            for (int64_t m = 0; m < len; ++m) HIP_TRY(c, adj_launch(b, len, A.cur, ring, m, c->stream));
            ring += (int)len;
        }
        A.cur = (A.cur + (int)len) & 1;
        HIP_TRY(c, hipEventRecord(A.ev_adj[b], c->stream));
    }
    if (ring > 0) HIP_TRY(c, lbm::launch_adjoint_reduce(part, ring, A.blocks, red, acc, c->stream));
    double sums[4];
    HIP_TRY(c, hipMemcpyAsync(sums, acc, sizeof sums, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // theta = (dp, a, b, T): g = dp/nx, RT = R T, a_eff = a alpha(T) (alpha = 1 for CS), b
    grad[0] = seed * sums[0] / c->nx;
    if (eos == LBM_EOS_CS) {
        grad[1] = seed * sums[2];
        grad[2] = seed * sums[3];
        grad[3] = seed * sums[1] * c->eos.R;
    } else {  // PR: alpha depends on T/Tc and Tc on (a, b); like the tangents, only dp and T
        grad[1] = NAN;
        grad[2] = NAN;
        grad[3] = seed * (sums[1] * c->eos.R + sums[2] * c->eos.a * pr_alpha_dT(c->p.omega, c->eos.T, c->eos.Tc));
    }
    A.seed = seed;
    A.swept = true;
    return LBM_OK;
}

lbm_status lbm_adjoint_state_gradient(lbm_ctx* c, double* dJ_df) {
    if (!c || !dJ_df) return LBM_EINVAL;
    lbm_ctx::Adjoint& A = c->adj;
    if (!A.bound || !A.swept) return fail(c, LBM_ESTATE, "lbm_adjoint_state_gradient needs lbm_adjoint_backward first");
    lbm::StepArgs a = make_args(c);
    double* g0 = reinterpret_cast<double*>(A.dev + A.off_g0);
    HIP_TRY(c, lbm::launch_adjoint_gather(A.dev + A.off_lam[A.cur], a, c->p.storage, g0, c->stream));
    const size_t n = (size_t)9 * c->nx * c->ny;
    HIP_TRY(c, hipMemcpyAsync(dJ_df, g0, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < n; ++i) dJ_df[i] *= A.seed;
    return LBM_OK;
}

lbm_status lbm_components(lbm_ctx* c, double threshold, int connectivity, lbm_component* out, int64_t cap,
                          int64_t* n_out, lbm_aerosol_summary* summary) {
    if (!c) return LBM_EINVAL;
    if (!c->initialized) return fail(c, LBM_ESTATE, "not initialised");
    if (std::isnan(threshold)) threshold = 0.5 * (c->rho_g + c->rho_l);
    if (std::isnan(threshold)) return fail(c, LBM_EINVAL, "no coexistence densities above Tc: give a threshold");
    if (lbm_status st = ensure_fields(c)) return st;
    std::vector<double> rho((size_t)c->nx * c->ny);
    HIP_TRY(c, hipMemcpyAsync(rho.data(), c->dev + c->off_rho, rho.size() * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const double rho_g = std::isnan(c->rho_g) ? 0.0 : c->rho_g;
    lbm_status s = lbm::label_components(rho.data(), c->nx, c->ny, c->p.x_periodic == 1, c->p.y_periodic == 1,
                                         threshold, rho_g, connectivity, out, cap, n_out, summary);
    if (s) return fail(c, s, "lbm_components: connectivity must be 4 or 8 and cap >= 0");
    if (summary) summary->step = c->steps;
    return LBM_OK;
}

// ---- checkpoint / resume ---------------------------------------------------------
//
// File: the 8-byte magic "LBMCKPT1", then the fields below in this order (native
// byte order, as the library's own structs), then the current distribution
// buffer [9][ny][pitch] in the storage type and the emitted fields rho, vx, vy
// [ny][nx] FP64, then an FNV-1a 64-bit hash of every preceding byte.
namespace {
constexpr char kCkptMagic[8] = {'L', 'B', 'M', 'C', 'K', 'P', 'T', '1'};
struct CkptHeader {
    int32_t nx, ny;
    double tau;
    lbm_params p;
    int64_t steps;
    lbm_check_result check;
    double acc[lbm::kWallAccVals];  // time integrals and running extremes of the wall stresses
    double dtheta[4];               // F64T tangent direction
    uint32_t sr;                    // F16R: counter of the next step
    uint32_t pad;
    uint64_t f_bytes;
};
struct Fnv64 {
    uint64_t h = 14695981039346656037ull;  // the 64-bit FNV offset basis
    void add(const void* p, size_t n) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    }
};
bool params_equal(const lbm_params& a, const lbm_params& b) {
    // field by field (the struct has padding); NaN defaults compare equal
    auto same = [](double x, double y) { return x == y || (std::isnan(x) && std::isnan(y)); };
    return a.eos == b.eos && same(a.a, b.a) && same(a.b, b.b) && same(a.R, b.R) && same(a.omega, b.omega) &&
           same(a.T_over_Tc, b.T_over_Tc) && same(a.k, b.k) && same(a.kappa, b.kappa) && same(a.s_e, b.s_e) &&
           same(a.s_eps, b.s_eps) && same(a.s_q, b.s_q) && same(a.s_j, b.s_j) && same(a.rho_wall, b.rho_wall) &&
           same(a.dp, b.dp) && a.x_periodic == b.x_periodic && a.y_periodic == b.y_periodic &&
           a.storage == b.storage && same(a.rho0_shift, b.rho0_shift) && same(a.v_limit, b.v_limit);
}
}  // namespace

lbm_status lbm_save(lbm_ctx* c, const char* path) {
    if (!c || !path) return LBM_EINVAL;
    if (!c->bound || !c->initialized) return fail(c, LBM_ESTATE, "lbm_save needs an initialised lattice");
    if (c->in_batch) return fail(c, LBM_ESTATE, "a batch case is not saved on its own");
    lbm_status st = flush_wall(c);  // the accumulators then hold every step so far
    if (st) return st;
    st = ensure_fields(c);
    if (st) return st;
    CkptHeader h{};
    h.nx = c->nx;
    h.ny = c->ny;
    h.tau = c->tau;
    h.p = c->p;
    h.steps = c->steps;
    h.check = c->check;
    for (int q = 0; q < 4; ++q) h.dtheta[q] = c->dtheta[q];
    h.f_bytes = (uint64_t)c->plane * 9 * storage_bytes(c->p.storage);
    const size_t nxy = (size_t)c->nx * c->ny;
    std::vector<unsigned char> f((size_t)h.f_bytes);
    std::vector<double> fields(3 * nxy);
    uint32_t sr[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(h.acc, c->dev + c->off_acc, sizeof h.acc, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(sr, c->dev + c->off_sr, sizeof sr, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(f.data(), c->dev + c->off_f[c->cur], f.size(), hipMemcpyDeviceToHost, c->stream));
    const size_t off_fields[3] = {c->off_rho, c->off_vx, c->off_vy};
    for (int q = 0; q < 3; ++q)
        HIP_TRY(c, hipMemcpyAsync(fields.data() + q * nxy, c->dev + off_fields[q], nxy * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    h.sr = sr[c->cur];
    Fnv64 hash;
    hash.add(kCkptMagic, sizeof kCkptMagic);
    hash.add(&h, sizeof h);
    hash.add(f.data(), f.size());
    hash.add(fields.data(), fields.size() * sizeof(double));
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return fail(c, LBM_EINVAL, "lbm_save: cannot open %s for writing", path);
    bool ok = std::fwrite(kCkptMagic, sizeof kCkptMagic, 1, fp) == 1 && std::fwrite(&h, sizeof h, 1, fp) == 1 &&
              std::fwrite(f.data(), 1, f.size(), fp) == f.size() &&
              std::fwrite(fields.data(), sizeof(double), fields.size(), fp) == fields.size() &&
              std::fwrite(&hash.h, sizeof hash.h, 1, fp) == 1;
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok) return fail(c, LBM_EINVAL, "lbm_save: writing %s failed", path);
    return LBM_OK;
}

lbm_status lbm_load(lbm_ctx* c, const char* path) {
    if (!c || !path) return LBM_EINVAL;
    if (!c->bound) return fail(c, LBM_ESTATE, "lbm_bind must come first");
    if (c->in_batch) return fail(c, LBM_ESTATE, "a batch case is not loaded on its own");
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return fail(c, LBM_EINVAL, "lbm_load: cannot open %s", path);
    char magic[8];
    CkptHeader h{};
    bool ok = std::fread(magic, sizeof magic, 1, fp) == 1 && std::memcmp(magic, kCkptMagic, sizeof magic) == 0 &&
              std::fread(&h, sizeof h, 1, fp) == 1;
    const size_t nxy = (size_t)c->nx * c->ny;
    const uint64_t f_bytes = (uint64_t)c->plane * 9 * storage_bytes(c->p.storage);
    ok = ok && h.nx == c->nx && h.ny == c->ny && h.tau == c->tau && h.f_bytes == f_bytes && params_equal(h.p, c->p);
    std::vector<unsigned char> f;
    std::vector<double> fields;
    uint64_t stored = 0;
    if (ok) {
        f.resize((size_t)f_bytes);
        fields.resize(3 * nxy);
        ok = std::fread(f.data(), 1, f.size(), fp) == f.size() &&
             std::fread(fields.data(), sizeof(double), fields.size(), fp) == fields.size() &&
             std::fread(&stored, sizeof stored, 1, fp) == 1;
    }
    std::fclose(fp);
    if (!ok)
        return fail(c, LBM_EINVAL, "lbm_load: %s is not a checkpoint of a lattice with these sizes, tau and "
                                   "parameters", path);
    Fnv64 hash;
    hash.add(kCkptMagic, sizeof kCkptMagic);
    hash.add(&h, sizeof h);
    hash.add(f.data(), f.size());
    hash.add(fields.data(), fields.size() * sizeof(double));
    if (hash.h != stored) return fail(c, LBM_EINVAL, "lbm_load: %s is corrupt (hash mismatch)", path);
    c->cur = 0;
    const uint32_t sr[2] = {h.sr, 0};
    HIP_TRY(c, hipMemcpyAsync(c->dev + c->off_f[0], f.data(), f.size(), hipMemcpyHostToDevice, c->stream));
    const size_t off_fields[3] = {c->off_rho, c->off_vx, c->off_vy};
    for (int q = 0; q < 3; ++q)
        HIP_TRY(c, hipMemcpyAsync(c->dev + off_fields[q], fields.data() + q * nxy, nxy * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->dev + c->off_acc, h.acc, sizeof h.acc, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, lbm::launch_fill(c->at<double>(c->off_acc) + lbm::kAccTicket, 0.0, 1, c->stream));
    HIP_TRY(c, lbm::launch_fill(c->at<double>(c->off_acc) + lbm::kAccNextStep, double(h.steps + 1), 1, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->dev + c->off_sr, sr, sizeof sr, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->steps = h.steps;
    c->fields_step = h.steps;
    c->prev_valid = false;
    c->check = h.check;
    for (int q = 0; q < 4; ++q) c->dtheta[q] = h.dtheta[q];
    c->graphs.drop();  // the tangent direction is part of the captured launches
    c->ring_fill = 0;
    c->last_slot = -1;
    c->ring_first_step = h.steps + 1;
    c->hist_first = h.steps + 1;
    c->initialized = true;
    c->adj.recorded = c->adj.swept = false;
    return LBM_OK;
}

lbm_status lbm_fields_device(lbm_ctx* c, void* rho, void* vx, void* vy, int fp64) {
    if (!c) return LBM_EINVAL;
    if (!c->initialized) return fail(c, LBM_ESTATE, "not initialised");
    const long long n = (long long)c->nx * c->ny;
    void* outs[3] = {rho, vx, vy};
    const size_t off_fields[3] = {c->off_rho, c->off_vx, c->off_vy};
    const size_t elem = fp64 ? sizeof(double) : sizeof(float);
    for (int q = 0; q < 3; ++q) {
        if (!outs[q]) continue;
        if (reinterpret_cast<uintptr_t>(outs[q]) % elem)
            return fail(c, LBM_EINVAL, "fields_device: output %d is not aligned to its element size", q);
        const char* why = nullptr;
        if (lbm_status st = device_range_check(outs[q], (size_t)n * elem, &why))
            return fail(c, st, "fields_device: output %d: %s", q, why);
    }
    if (lbm_status st = ensure_fields(c)) return st;
    for (int q = 0; q < 3; ++q) {
        if (!outs[q]) continue;
        const double* src = c->at<double>(off_fields[q]);
        if (fp64)
            HIP_TRY(c, hipMemcpyAsync(outs[q], src, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        else
            HIP_TRY(c, lbm::launch_to_f32(src, static_cast<float*>(outs[q]), n, c->stream));
    }
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
    if (c && c->in_batch) return;  // owned by its batch (lbm_batch_destroy frees it)
    delete c;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: many independent lattices advanced by one kernel launch per step.

namespace {
// Output rows of the two-step tiles for a storage type, 0 where it has no two-step kernel.
int batch_tile2_rows(int storage) {
    switch (storage) {
        case LBM_F64:
        case LBM_F32D: return lbm::kTile2RowsF64;
        case LBM_F32:
        case LBM_F16S:
        case LBM_BF16S:
        case LBM_F32S: return lbm::kTile2Rows;
        default: return 0;
    }
}
}  // namespace

struct lbm_batch {
    StepGraphs graphs;
    std::vector<lbm_ctx*> cases;
    std::vector<int> tile_start;   // ncases + 1
    std::vector<int> tile_start2;  // the same for the two-step tiles
    int L = 1;                     // steps per launch (2: the two-step kernel)
    size_t off_desc = 0, off_tiles = 0, off_tiles2 = 0, off_flush = 0, total = 0;
    int nflush = 0;  // cases with walls (their wall rings are reduced together)
    std::vector<size_t> off_case;
    char* dev = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    std::string err;
    ~lbm_batch() {
        for (lbm_ctx* c : cases) delete c;
    }
};

namespace {

lbm_status bfail(lbm_batch* b, lbm_status s, const std::string& msg) {
    if (b) b->err = msg;
    return s;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_create(int n, const int* nx, const int* ny, const double* tau, const lbm_params* params,
                            lbm_batch** out) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (n < 1 || !nx || !ny || !tau || !params) return LBM_EINVAL;
    auto* b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_ENOMEM;
    const lbm_params& p0 = params[0];
    for (int k = 0; k < n; ++k) {
        const lbm_params& p = params[k];
        // one kernel instance serves every case: storage, EOS kind and tile shape agree, and the
        // cases are checked together
        if (p.storage != p0.storage || p.storage == LBM_F64T || p.eos != p0.eos || p.schedule != lbm::kScheduleTile ||
            p.tile_rows != p0.tile_rows || p.tile_waves != p0.tile_waves || p.check_every != p0.check_every ||
            p.graph_steps != p0.graph_steps || p.fused_steps != p0.fused_steps) {
            delete b;
            return LBM_EINVAL;
        }
        lbm_ctx* c = nullptr;
        lbm_status s = lbm_create(nx[k], ny[k], tau[k], &p, &c);
        if (s) {
            delete b;
            return s;
        }
        c->in_batch = true;
        b->cases.push_back(c);
    }
    size_t o = 0;
    b->off_desc = o; o += align256((size_t)n * sizeof(lbm::StepArgs));
    b->off_tiles = o; o += align256((size_t)(n + 1) * sizeof(int));
    b->off_tiles2 = o; o += align256((size_t)(n + 1) * sizeof(int));
    b->off_flush = o; o += align256((size_t)n * sizeof(lbm::WallFlush));
    const int rows2 = batch_tile2_rows(p0.storage);
    b->L = (rows2 > 0 && p0.fused_steps == 2) ? 2 : 1;
    long long tiles2 = 0;
    int tiles = 0;
    for (int k = 0; k < n; ++k) {
        lbm_ctx* c = b->cases[k];
        b->off_case.push_back(o);
        o += align256(c->total);
        b->tile_start.push_back(tiles);
        b->tile_start2.push_back((int)tiles2);
        const long long t = (long long)tiles + (long long)c->nstrip * ((c->ny + c->ty - 1) / c->ty);
        tiles2 += rows2 > 0 ? lbm::tiles2(c->nx, c->ny, rows2) : 0;
        if (t > (1LL << 30) || tiles2 > (1LL << 30)) {
            delete b;
            return LBM_EINVAL;
        }
        tiles = (int)t;
    }
    b->tile_start.push_back(tiles);
    b->tile_start2.push_back((int)tiles2);
    b->total = o;
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_workspace(const lbm_batch* b, size_t* bytes) {
    if (!b || !bytes) return LBM_EINVAL;
    *bytes = b->total;
    return LBM_OK;
}

lbm_status lbm_batch_bind(lbm_batch* b, void* device_ptr, size_t bytes, void* hip_stream) {
    if (!b) return LBM_EINVAL;
    if (!device_ptr || (reinterpret_cast<uintptr_t>(device_ptr) & 255))
        return bfail(b, LBM_EINVAL, "workspace pointer must be non-null and 256-byte aligned");
    if (bytes < b->total) return bfail(b, LBM_ENOMEM, "workspace too small for the batch");
    const char* why = nullptr;
    if (lbm_status st = device_range_check(device_ptr, b->total, &why))
        return bfail(b, st, std::string("workspace: ") + why);
    b->dev = static_cast<char*>(device_ptr);
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->graphs.drop();
    std::vector<lbm::StepArgs> desc;
    for (size_t k = 0; k < b->cases.size(); ++k) {
        lbm_ctx* c = b->cases[k];
        c->in_batch = false;  // lbm_bind is shared with single contexts
        lbm_status s = lbm_bind(c, b->dev + b->off_case[k], c->total, hip_stream);
        c->in_batch = true;
        if (s) return bfail(b, s, "case " + std::to_string(k) + ": " + c->err);
        lbm::StepArgs a = make_args(c);
        a.fin = c->dev + c->off_f[0];
        a.fout = c->dev + c->off_f[1];
        desc.push_back(a);
    }
    std::vector<lbm::WallFlush> flush;
    for (lbm_ctx* c : b->cases)
        if (!c->p.y_periodic)
            flush.push_back(lbm::WallFlush{c->at<double>(c->off_ring), c->nx, c->at<lbm_stress_summary>(c->off_hist),
                                           c->p.history_cap, c->at<double>(c->off_wscr), c->at<double>(c->off_acc)});
    b->nflush = (int)flush.size();
    hipError_t e = hipMemcpyAsync(b->dev + b->off_desc, desc.data(), desc.size() * sizeof(lbm::StepArgs),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !flush.empty())
        e = hipMemcpyAsync(b->dev + b->off_flush, flush.data(), flush.size() * sizeof(lbm::WallFlush),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->dev + b->off_tiles, b->tile_start.data(), b->tile_start.size() * sizeof(int),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->dev + b->off_tiles2, b->tile_start2.data(), b->tile_start2.size() * sizeof(int),
                           hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("batch descriptors: ") + hipGetErrorString(e));
    b->bound = true;
    return LBM_OK;
}

lbm_status lbm_batch_case(lbm_batch* b, int k, lbm_ctx** ctx) {
    if (!b || !ctx || k < 0 || k >= (int)b->cases.size()) return LBM_EINVAL;
    *ctx = b->cases[(size_t)k];
    return LBM_OK;
}

namespace {

// n steps of every case, or (dry) only the capture of the graphs they would replay; as
// step_impl for one lattice: checks (with one wait for all cases) at multiples of the check
// cadence, graphs in between, and the cases' wall rings reduced on the stream at the end.
lbm_status batch_step_impl(lbm_batch* b, int64_t n, int* failed_case, bool dry) {
    lbm_ctx* c0 = b->cases[0];
    for (lbm_ctx* c : b->cases) {
        if (!c->initialized) return bfail(b, LBM_ESTATE, "every case must be initialised before stepping");
        if (c->steps != c0->steps || c->cur != c0->cur || c->ring_fill != c0->ring_fill)
            return bfail(b, LBM_ESTATE, "the cases must be initialised together (equal step counts)");
    }
    struct Cursor {
        int cur, ring_fill, last_slot;
        int64_t steps, ring_first_step;
    };
    std::vector<Cursor> saved;
    for (lbm_ctx* c : b->cases) saved.push_back({c->cur, c->ring_fill, c->last_slot, c->steps, c->ring_first_step});
    const int ncases = (int)b->cases.size();
    const auto* desc = reinterpret_cast<const lbm::StepArgs*>(b->dev + b->off_desc);
    const auto* tiles = reinterpret_cast<const int*>(b->dev + b->off_tiles);
    const auto* tiles2 = reinterpret_cast<const int*>(b->dev + b->off_tiles2);
    const int G = c0->graph_steps();
    const int L = b->L;  // steps per launch; G is a multiple of it
    auto advance = [&](int nsteps, int launches) {  // each launch flips the buffers once
        for (lbm_ctx* c : b->cases) {
            c->cur = (c->cur + launches) & 1;
            c->last_slot = c->ring_fill + nsteps - 1;
            c->ring_fill += nsteps;
            c->steps += nsteps;
        }
    };
    // one launch of `steps` (1 or 2) steps of every case from buffer parity `par`, wall arrays from ring slot `slot`
    auto launch_any = [&](int steps, int par, int slot, bool emit, hipStream_t s) -> hipError_t {
        if (steps == 2)
            return lbm::launch_step2_batch(desc, tiles2, ncases, b->tile_start2.back(), par, slot, c0->p.storage,
                                           c0->p.eos, emit, s);
        return lbm::launch_step_batch(desc, tiles, ncases, b->tile_start.back(), par, slot, c0->p.storage, c0->p.eos,
                                      c0->ty, c0->tile_waves, emit, s);
    };
    auto flush_all = [&]() -> lbm_status {  // every case's wall ring in one pair of launches
        if (c0->ring_fill == 0) return LBM_OK;
        if (!dry) {
            hipError_t e = lbm::launch_wall_reduce_batch(reinterpret_cast<const lbm::WallFlush*>(b->dev + b->off_flush),
                                                         b->nflush, c0->ring_fill, b->stream);
            if (e != hipSuccess)
                return bfail(b, LBM_EDEVICE, std::string("batch wall reduce: ") + hipGetErrorString(e));
        }
        for (lbm_ctx* c : b->cases) {
            c->ring_first_step += c->ring_fill;
            c->ring_fill = 0;
        }
        return LBM_OK;
    };
    auto launch_direct = [&](int steps, bool emit) -> lbm_status {
        if (c0->ring_fill + steps > kRingCap) {
            lbm_status s = flush_all();
            if (s) return s;
        }
        if (!dry) {
            hipError_t e = launch_any(steps, c0->cur, c0->ring_fill, emit, b->stream);
            if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("batch step: ") + hipGetErrorString(e));
        }
        advance(steps, 1);
        return LBM_OK;
    };
    int64_t done = 0;
    while (done < n) {
        const int64_t next_check = (c0->steps / c0->p.check_every + 1) * c0->p.check_every;
        const int64_t seg = std::min<int64_t>(n - done, next_check - c0->steps);
        const bool check = c0->steps + seg == next_check;
        // the step that emits for a check, and with two steps per launch the last step of
        // the call, are one-step launches
        const int64_t tail = (check || L == 2) ? 1 : 0;
        int64_t body = seg - tail;
        while (body > 0) {
            int m = G > 0 ? (int)std::min<int64_t>(body, G) : 0;
            if (L == 2) m &= ~1;
            hipGraphExec_t* ge = nullptr;
            if (m > 0) {
                if (c0->ring_fill + m > kRingCap) {
                    lbm_status s = flush_all();
                    if (s) return s;
                }
                ge = b->graphs.entry(c0->cur, c0->ring_fill, m, G, false);
            }
            if (!ge) {  // no graphs, or the cache of short runs is full: L steps per launch while they fit
                const int64_t mm = m > 0 ? m : body;
                for (int64_t k = 0; k < mm;) {
                    const int st = (L == 2 && mm - k >= 2) ? 2 : 1;
                    lbm_status s = launch_direct(st, false);
                    if (s) return s;
                    k += st;
                }
                body -= mm;
                continue;
            }
            const int nl = m / L;  // launches in the graph
            if (!*ge) {
                const int par = c0->cur, fill0 = c0->ring_fill;
                auto launch = [&](int j, hipStream_t s) { return launch_any(L, (par + j) & 1, fill0 + L * j, false, s); };
                hipError_t e = capture_graph(b->graphs, nl, launch, ge);
                if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("batch graph: ") + hipGetErrorString(e));
            }
            if (!dry) {
                hipError_t e = hipGraphLaunch(*ge, b->stream);
                if (e != hipSuccess)
                    return bfail(b, LBM_EDEVICE, std::string("batch graph launch: ") + hipGetErrorString(e));
            }
            advance(m, nl);
            body -= m;
        }
        if (tail) {
            lbm_status s = launch_direct(1, check);
            if (s) return s;
        }
        done += seg;
        if (!dry)
            for (lbm_ctx* c : b->cases) {
                c->prev_valid = true;
                if (check) c->fields_step = c->steps;
            }
        if (!check) break;
        lbm_status fs = flush_all();
        if (fs) return fs;
        if (dry) continue;
        // every case's check queued on the batch stream, one wait, then the host halves in case order
        for (int k = 0; k < ncases; ++k) {
            lbm_status s = check_launch(b->cases[(size_t)k]);
            if (s) return bfail(b, s, "case " + std::to_string(k) + ": " + b->cases[(size_t)k]->err);
        }
        if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, LBM_EDEVICE, "batch check: stream error");
        for (int k = 0; k < ncases; ++k) {
            lbm_status s = check_finish(b->cases[(size_t)k]);
            if (s) {
                if (failed_case) *failed_case = k;
                return bfail(b, s, "case " + std::to_string(k) + ": " + b->cases[(size_t)k]->err);
            }
        }
    }
    if (dry) {
        for (size_t k = 0; k < b->cases.size(); ++k) {
            lbm_ctx* c = b->cases[k];
            c->cur = saved[k].cur;
            c->ring_fill = saved[k].ring_fill;
            c->last_slot = saved[k].last_slot;
            c->steps = saved[k].steps;
            c->ring_first_step = saved[k].ring_first_step;
        }
        return LBM_OK;
    }
    lbm_status fs = flush_all();  // queued, as for one lattice
    if (fs) return fs;
    for (int k = 0; k < ncases; ++k)
        if (b->cases[(size_t)k]->check.unstable_step >= 0) {
            if (failed_case) *failed_case = k;
            return bfail(b, LBM_EUNSTABLE, "case " + std::to_string(k) + ": unstable since step " +
                                               std::to_string(b->cases[(size_t)k]->check.unstable_step));
        }
    return LBM_OK;
}

}  // namespace

lbm_status lbm_batch_step(lbm_batch* b, int64_t n, int* failed_case) {
    if (failed_case) *failed_case = -1;
    if (!b || n < 0) return LBM_EINVAL;
    if (!b->bound) return bfail(b, LBM_ESTATE, "lbm_batch_bind must come first");
    return batch_step_impl(b, n, failed_case, false);
}

lbm_status lbm_batch_capture(lbm_batch* b, int64_t n) {
    if (!b || n < 0) return LBM_EINVAL;
    if (!b->bound) return bfail(b, LBM_ESTATE, "lbm_batch_bind must come first");
    return batch_step_impl(b, n, nullptr, true);
}

lbm_status lbm_batch_autotune(lbm_batch* b, int trial_steps, int* tile_rows, int* tile_waves, double* us_per_step) {
    if (!b || trial_steps < 1) return LBM_EINVAL;
    if (!b->bound) return bfail(b, LBM_ESTATE, "lbm_batch_bind must come first");
    lbm_ctx* c0 = b->cases[0];
    for (lbm_ctx* c : b->cases) {
        if (!c->initialized) return bfail(b, LBM_ESTATE, "every case must be initialised before tuning");
        lbm_status s = flush_wall(c);
        if (s) return bfail(b, s, c->err);
        s = ensure_fields(c);  // the trials overwrite the latest step's input
        if (s) return bfail(b, s, c->err);
        c->prev_valid = false;
    }
    const int ncases = (int)b->cases.size();
    // trial launch table: each case's diagnostics redirected into its (flushed) wall ring
    std::vector<lbm::StepArgs> trial, real;
    for (lbm_ctx* c : b->cases) {
        lbm::StepArgs a = trial_args(c);
        a.fin = c->dev + c->off_f[0];
        a.fout = c->dev + c->off_f[1];
        trial.push_back(a);
        lbm::StepArgs r = make_args(c);
        r.fin = a.fin;
        r.fout = a.fout;
        real.push_back(r);
    }
    auto* desc = reinterpret_cast<lbm::StepArgs*>(b->dev + b->off_desc);
    const auto* tiles = reinterpret_cast<const int*>(b->dev + b->off_tiles);
    const size_t bytes = trial.size() * sizeof(lbm::StepArgs);
    hipError_t e = hipMemcpyAsync(desc, trial.data(), bytes, hipMemcpyHostToDevice, b->stream);
    double best = INFINITY;
    TileShape pick = {c0->ty, c0->tile_waves};
    std::vector<std::vector<int>> starts;  // host sources of the copies stay alive until the final synchronisation
    for (const TileShape& t : kTileShapes) {
        if (e != hipSuccess) break;
        double us = 0;
        // the tile count of a shape differs: one launch of every case's tiles for this shape
        starts.emplace_back(1, 0);
        std::vector<int>& start = starts.back();
        for (lbm_ctx* c : b->cases) start.push_back(start.back() + c->nstrip * ((c->ny + t.rows - 1) / t.rows));
        // the per-case first-tile table lives after the descriptors; keep the real one and restore it below
        e = hipMemcpyAsync(const_cast<int*>(tiles), start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice,
                           b->stream);
        if (e != hipSuccess) break;
        e = time_launches(b->stream, trial_steps, [&] {  // wall arrays to a slot other than the latest step's
            return lbm::launch_step_batch(desc, tiles, ncases, start.back(), c0->cur, (c0->last_slot + 1) % kRingCap,
                                          c0->p.storage, c0->p.eos, t.rows, t.waves, false, b->stream);
        }, &us);
        if (e == hipSuccess && us < best) { best = us; pick = t; }
    }
    // two steps per launch, where the storage has the two-step kernel (its own tile table);
    // the two wall arrays go to two consecutive ring slots, neither of them the latest step's
    int fused = 1;
    if (e == hipSuccess && batch_tile2_rows(c0->p.storage) > 0) {
        double us = 0;
        const int slot = c0->last_slot + 1 <= kRingCap - 2 ? c0->last_slot + 1 : 0;
        const auto* tiles2 = reinterpret_cast<const int*>(b->dev + b->off_tiles2);
        e = time_launches(b->stream, (trial_steps + 1) / 2, [&] {
            return lbm::launch_step2_batch(desc, tiles2, ncases, b->tile_start2.back(), c0->cur, slot, c0->p.storage,
                                           c0->p.eos, false, b->stream);
        }, &us);
        if (e == hipSuccess && 0.5 * us < best) {
            best = 0.5 * us;
            fused = 2;
        }
    }
    // the chosen shape's tile table and the real launch table
    starts.emplace_back(1, 0);
    std::vector<int>& start = starts.back();
    for (lbm_ctx* c : b->cases) start.push_back(start.back() + c->nstrip * ((c->ny + pick.rows - 1) / pick.rows));
    if (e == hipSuccess) e = hipMemcpyAsync(desc, real.data(), bytes, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(const_cast<int*>(tiles), start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, LBM_EDEVICE, std::string("batch autotune: ") + hipGetErrorString(e));
    b->tile_start = start;
    b->L = fused;
    for (lbm_ctx* c : b->cases) {
        c->ty = c->p.tile_rows = pick.rows;
        c->tile_waves = c->p.tile_waves = pick.waves;
        c->p.fused_steps = fused;
        c->nchunk = std::max(1, c->ny / c->ty);
    }
    b->graphs.drop();
    if (tile_rows) *tile_rows = pick.rows;
    if (tile_waves) *tile_waves = pick.waves;
    if (us_per_step) *us_per_step = best;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) { delete b; }

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
