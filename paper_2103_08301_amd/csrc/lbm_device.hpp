// lbm_device.hpp -- device code of the EOS-based multiphase MRT lattice
// Boltzmann step (arXiv 2103.08301, Sec. 2), shared by the HIP translation
// units of the library: one unit per storage type instantiates the step
// kernels for that type, so the units compile in parallel.  Everything here
// has internal linkage; the units export plain launch functions declared in
// lbm_internal.hpp.
//
// The step is one fused kernel.  In the row-march schedule each 64-lane
// wavefront owns a strip of 64 consecutive columns (60 output columns plus a
// 2-column halo on each side) and a chunk of rows, and marches up the chunk
// one row at a time:
//
//   row r     : pull-stream the 9 populations (structure-of-arrays loads that
//               are coalesced along x), density, EOS field phi(rho)
//   row r - 1 : Laplacian of rho and gradients of phi (and of rho on the wall
//               rows), from the three most recent rows kept in registers and
//               their x-neighbours exchanged across lanes
//   row r - 2 : gradient of the Laplacian, force of eq. 2.17, velocity shift,
//               MRT collision, store, wall diagnostics
//
// so the density and EOS field never leave registers: the only global traffic
// per node and step is reading 9 and writing 9 populations (plus the halo rows
// and columns, which the neighbouring strips also read).  The tile schedules
// below keep the same fields in LDS instead.  No MFMA: the update is a
// bandwidth-bound stencil, not a dense contraction.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "lbm_internal.hpp"

namespace lbm {
namespace {

// D2Q9: e0=(0,0) e1=(1,0) e2=(0,1) e3=(-1,0) e4=(0,-1) e5=(1,1) e6=(-1,1) e7=(-1,-1) e8=(1,-1)
__host__ __device__ constexpr int ex(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int ey(int i) {
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i < 5 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5); }
static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opposites");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opposites");
template <class C>
__host__ __device__ constexpr C wgt(int i) {
    return i == 0 ? C(4) / C(9) : (i < 5 ? C(1) / C(9) : C(1) / C(36));
}
// 9 w_i: the shifted codecs' multipliers of the shift unit (powers of two, exact).
template <class C>
__host__ __device__ constexpr C kwt(int i) {
    return i == 0 ? C(4) : (i < 5 ? C(1) : C(0.25));
}

__device__ inline int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}
__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ---------------------------------------------------------------------------
// Storage codecs.

struct CodecF64 {
    using S = double;
    using C = double;
    static constexpr bool kShifted = false;
    template <int I>
    __device__ static C work(C f, C) { return f; }
    template <int I>
    __device__ static C decode(S s, C) { return s; }
    template <int I>
    __device__ static C load(const S* p, C r) { return decode<I>(*p, r); }
    template <int I>
    __device__ static S encode(C v, C) { return v; }
    template <int I>
    __device__ static void store(S* p, C v, C r) { *p = encode<I>(v, r); }
};

struct CodecF32 {
    using S = float;
    using C = float;
    static constexpr bool kShifted = false;
    template <int I>
    __device__ static C work(C f, C) { return f; }
    template <int I>
    __device__ static C decode(S s, C) { return s; }
    template <int I>
    __device__ static C load(const S* p, C r) { return decode<I>(*p, r); }
    template <int I>
    __device__ static S encode(C v, C) { return v; }
    template <int I>
    __device__ static void store(S* p, C v, C r) { *p = encode<I>(v, r); }
};

// FP32 storage, FP64 arithmetic (same bytes per node as FP32).
struct CodecF32D {
    using S = float;
    using C = double;
    static constexpr bool kShifted = false;
    template <int I>
    __device__ static C work(C f, C) { return f; }
    template <int I>
    __device__ static C decode(S s, C) { return double(s); }
    template <int I>
    __device__ static C load(const S* p, C r) { return decode<I>(*p, r); }
    template <int I>
    __device__ static S encode(C v, C) { return float(v); }
    template <int I>
    __device__ static void store(S* p, C v, C r) { *p = encode<I>(v, r); }
};

// The shifted codecs below store the deviations d_i = f_i - k_i q, with
// k_i = 9 w_i in {4, 1, 1/4} and the shift unit q = rho0 / 9 on a grid of 2^-24
// (the host rounds it), passed in place of rho0.  The kernels compute with the
// deviations themselves (their working values): the shifts k_i q have the
// moments of a fluid at rest with density 9q, so rho = sum d_i + 9q, the momenta
// and the other non-energy moments of d equal those of f, and the collision's
// energy terms pair the moments of d with rho - 9q (node_rho, moment_rho, below).
// A load is then a plain conversion and a store one rounding, with no shift to
// add back and take off at every node; work() forms d_i from a full f_i (the
// initialisation).  9q is a multiple of 2^-24, exact in FP32 below 1; above, its
// FP32 rounding is smaller than that of rho itself.

// FP32 storage of f_i - k_i q, FP32 arithmetic.
struct CodecF32S {
    using S = float;
    using C = float;
    static constexpr bool kShifted = true;
    template <int I>
    __device__ static C work(C f, C q) { return __builtin_fmaf(-kwt<float>(I), q, f); }
    template <int I>
    __device__ static C decode(S s, C) { return s; }
    template <int I>
    __device__ static C load(const S* p, C q) { return decode<I>(*p, q); }
    template <int I>
    __device__ static S encode(C v, C) { return v; }
    template <int I>
    __device__ static void store(S* p, C v, C q) { *p = encode<I>(v, q); }
};

// FP16 storage of f_i - k_i q, FP32 arithmetic, round-to-nearest-even.
struct CodecF16S {
    using S = _Float16;
    using C = float;
    static constexpr bool kShifted = true;
    template <int I>
    __device__ static C work(C f, C q) { return __builtin_fmaf(-kwt<float>(I), q, f); }
    template <int I>
    __device__ static C decode(S s, C) { return static_cast<float>(s); }
    template <int I>
    __device__ static C load(const S* p, C q) { return decode<I>(*p, q); }
    template <int I>
    __device__ static S encode(C v, C) { return static_cast<_Float16>(v); }
    template <int I>
    __device__ static void store(S* p, C v, C q) { *p = encode<I>(v, q); }
};

// Integer hash of 32 bits (Wellons' "lowbias32" from his hash-prospector search:
// two xorshift-multiply rounds and a final xorshift).
__device__ inline uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Stochastic rounding of v to FP16 with gfx950's conversion instruction
// (v_cvt_sr_f16_f32): it rounds |v| up to the next FP16 value when t + r/2^32 >= 1,
// t the fraction of the FP16 spacing by which |v| exceeds the FP16 value below it
// and r the random operand, so with r uniform over 32 bits the chance of rounding
// up is t and the expected rounding error is zero.  (Measured on the device with
// the top 13 bits of r swept exhaustively: the fraction rounded up equals t for
// normals, values just above and below powers of two, negative values and FP16
// subnormals, every result is one of v's two FP16 neighbours, and the low 13 bits
// of r decide only near-ties.)
__device__ inline _Float16 f16_stochastic(float v, uint32_t r) {
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    half2_t z = {};
    z = __builtin_amdgcn_cvt_sr_f16_f32(z, v, r, false);
    return z[0];
}

// The random word of population I: word I / 3 of the node's three hash words,
// rotated so that its bits 10 (I mod 3) .. 10 (I mod 3) + 9, drawn for this
// population alone, are the top bits that decide the rounding.  Every rotated word
// is uniform over 32 bits; populations sharing a hash word share only the low bits,
// which decide near-ties.
template <int I>
__device__ inline uint32_t sr_word(const uint32_t (&h)[3]) {
    return __builtin_amdgcn_alignbit(h[I / 3], h[I / 3], 10u * (I % 3) + 10u);
}

// FP16 storage of f_i - k_i q with stochastic rounding (the step kernel
// passes the random bits).  Round-to-nearest repeats the same error every step
// wherever the populations are steady, which adds up to a mass source; rounding
// up or down at random makes the errors average out instead.  encode (used by
// the initialisation) rounds to nearest.
struct CodecF16R : CodecF16S {
    template <int I>
    __device__ static S encode_sr(C v, C, uint32_t r) { return f16_stochastic(v, r); }
};
template <class CD>
constexpr bool stochastic_codec() { return false; }
template <>
constexpr bool stochastic_codec<CodecF16R>() { return true; }

// BF16 storage of f_i - k_i q, FP32 arithmetic, round-to-nearest-even.
struct CodecBF16S {
    using S = uint16_t;
    using C = float;
    static constexpr bool kShifted = true;
    template <int I>
    __device__ static C work(C f, C q) { return __builtin_fmaf(-kwt<float>(I), q, f); }
    template <int I>
    __device__ static C decode(S s, C) { return __uint_as_float(static_cast<uint32_t>(s) << 16); }
    template <int I>
    __device__ static C load(const S* p, C q) { return decode<I>(*p, q); }
    template <int I>
    __device__ static S encode(C v, C) {
        uint32_t u = __float_as_uint(v);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return static_cast<uint16_t>(u >> 16);
    }
    template <int I>
    __device__ static void store(S* p, C v, C q) { *p = encode<I>(v, q); }
};

// Density of a node from its nine working values: their sum, plus the 9q of the
// shifts where the working values are deviations (sum_i k_i = 9).
template <class CD>
__device__ inline typename CD::C node_rho(const typename CD::C (&f)[9], typename CD::C q) {
    using C = typename CD::C;
    const C s = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    if constexpr (CD::kShifted)
        return s + C(9) * q;
    else
        return s;
}
// The density that the moments of a node's working values pair with in the
// collision's energy terms: rho, or rho - 9q for deviations.
template <class CD>
__device__ inline typename CD::C moment_rho(typename CD::C rho, typename CD::C q) {
    using C = typename CD::C;
    if constexpr (CD::kShifted)
        return rho - C(9) * q;
    else
        return rho;
}

// ---------------------------------------------------------------------------
// Arithmetic helpers.

// Hardware reciprocal refined by one Newton step (error well below 1 ulp).
__device__ inline float recip(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}
__device__ inline double recip(double x) { return 1.0 / x; }

// A step coefficient in the arithmetic type: the FP64 value, or its FP32
// rounding made on the host (the same value a conversion here would give).
// ---------------------------------------------------------------------------
// Tangent-linear arithmetic: a value and its derivative along one direction of
// the parameters (dp, a, b, T).  Running the step in this type propagates the
// exact derivative of every quantity (forward-mode differentiation).
struct Dual {
    double v, d;
    Dual() = default;  // trivial, so LDS arrays of Dual need no constructor
    __device__ constexpr Dual(double x) : v(x), d(0) {}  // constants have no tangent
    __device__ constexpr Dual(double x, double dx) : v(x), d(dx) {}
    __device__ explicit operator double() const { return v; }
};
__device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ inline Dual& operator+=(Dual& a, Dual b) { return a = a + b; }
__device__ inline Dual& operator-=(Dual& a, Dual b) { return a = a - b; }
__device__ inline Dual recip(Dual a) {
    const double r = 1.0 / a.v;
    return Dual(r, -a.d * r * r);
}
__device__ inline double value_of(double x) { return x; }
__device__ inline double value_of(float x) { return x; }
__device__ inline double value_of(Dual x) { return x.v; }
__device__ inline double tangent_of(double) { return 0.0; }
__device__ inline double tangent_of(float) { return 0.0; }
__device__ inline double tangent_of(Dual x) { return x.d; }

template <class C>
__device__ inline C coef(double d, float f, double t);
template <>
__device__ inline double coef<double>(double d, float, double) { return d; }
template <>
__device__ inline float coef<float>(double, float f, double) { return f; }
template <>
__device__ inline Dual coef<Dual>(double d, float, double t) { return Dual(d, t); }
#define LBM_COEF(C, name) coef<C>(a.name, a.cf.name, a.ct.name)

template <>
__host__ __device__ inline Dual wgt<Dual>(int i) {
    return Dual(wgt<double>(i));
}

// FP64 value and FP64 tangent of each population (16 bytes), tangent-linear arithmetic.
struct CodecF64T {
    using S = Dual;
    using C = Dual;
    static constexpr bool kShifted = false;
    template <int I>
    __device__ static C work(C f, C) { return f; }
    template <int I>
    __device__ static C decode(S s, C) { return s; }
    template <int I>
    __device__ static C load(const S* p, C r) { return decode<I>(*p, r); }
    template <int I>
    __device__ static S encode(C v, C) { return v; }
    template <int I>
    __device__ static void store(S* p, C v, C r) { *p = encode<I>(v, r); }
};

// x-neighbours across the 64 lanes of a wave with DPP wave shifts (a VALU
// operand modifier, no LDS traffic): wave_shl:1 reads lane + 1 (column x + 1),
// wave_shr:1 reads lane - 1 (column x - 1).  The edge lanes keep their own value;
// they belong to the halo and their neighbours are never used.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;
template <int CTRL>
__device__ inline float dpp_move(float v) {
    const int i = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(i, i, CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = int(b & 0xffffffffLL), hi = int(b >> 32);
    const int nlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
    const int nhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)nhi << 32) | (unsigned)nlo));
}
template <class C>
__device__ inline C shfl_next(C v) { return dpp_move<kDppWaveShl1>(v); }
template <class C>
__device__ inline C shfl_prev(C v) { return dpp_move<kDppWaveShr1>(v); }

// FP64 reciprocal from the hardware estimate refined by two Newton steps: for the
// EOS denominators, which lie in (0, 1], as accurate as the division for what the
// FP32 kernels keep of it, at a fraction of its cost.
__device__ inline double recip_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// phi = k^2 p0(rho) - rho/3: the nonideal part of the pressure in mesh units (eq. 2.17).
// NR: the denominator through recip_nr (FP64 only) instead of a division.
template <int EOS, class C, bool NR = false>
__device__ inline C phi_of(C rho, C RT, C a_eff, C b, C k2) {
    auto inv = [](C v) {
        if constexpr (NR) return recip_nr(v);
        else return recip(v);
    };
    C p0;
    if (EOS == LBM_EOS_CS) {
        const C eta = C(0.25) * b * rho;
        const C num = C(1) + eta * (C(1) + eta * (C(1) - eta));
        const C d = C(1) - eta;
        p0 = rho * RT * num * inv(d * d * d) - a_eff * rho * rho;
    } else {
        const C d = C(1) - b * rho;
        const C q = C(1) + b * rho * (C(2) - b * rho);
        p0 = rho * (RT * q - a_eff * rho * d) * inv(d * q);
    }
    return k2 * p0 - rho * C(1.0 / 3.0);
}

// The type in which the EOS field phi is evaluated, kept between the phases and
// differentiated: the arithmetic type, except with FP32 storage and FP32 arithmetic,
// where it is FP64.  At an interface grad phi is ~1e-2 while the pressure-drop force is
// ~1e-7 per node; phi rounded to FP32 (|phi| up to ~0.07) puts ~5e-9 of noise into
// every gradient, fixed in time while the flow is steady, and on the 4096 x 512 channel
// that drifted rho from the FP64 solution by 1.9e-5 over 2000 steps.  In FP64 the same run
// stays at 7.3e-6, for 2.8% of the step.  FP16/BF16 storage rounds far more than that.
template <class CD>
using PhiT = std::conditional_t<std::is_same<typename CD::C, float>::value && sizeof(typename CD::S) == 4, double,
                                typename CD::C>;

// phi of one node for storage CD, in PhiT<CD>: in FP64 from the FP64 coefficients
// where PhiT is FP64 and the arithmetic FP32.
template <class CD, int EOS>
__device__ inline PhiT<CD> phi_field(typename CD::C rho, const StepArgs& a) {
    using C = typename CD::C;
    if constexpr (std::is_same<PhiT<CD>, C>::value)
        return phi_of<EOS, C>(rho, LBM_COEF(C, RT), LBM_COEF(C, a_eff), LBM_COEF(C, b), LBM_COEF(C, k2));
    else
        return phi_of<EOS, double, true>(double(rho), a.RT, a.a_eff, a.b, a.k2);
}

template <int EOS, class C>
__device__ inline C p0_of(C rho, C RT, C a_eff, C b) {
    return phi_of<EOS, C>(rho, RT, a_eff, b, C(1)) + rho * C(1.0 / 3.0);
}

template <class C>
struct Row3 {  // a field value at a column and its two x-neighbours
    C c, e, w;
};

template <class C>
__device__ inline Row3<C> with_neighbours(C v) {
    return Row3<C>{v, shfl_next(v), shfl_prev(v)};
}

// Isotropic D2Q9 operators on three consecutive rows (s = y-1, m = y, n = y+1):
// grad = 3 sum w_i e_i psi(x + e_i), lap = 6 sum w_i (psi(x + e_i) - psi(x)).
template <class C>
__device__ inline C lap3(const Row3<C>& s, const Row3<C>& m, const Row3<C>& n) {
    return C(2.0 / 3.0) * (m.e + m.w + n.c + s.c) + C(1.0 / 6.0) * (n.e + n.w + s.e + s.w) - C(10.0 / 3.0) * m.c;
}
// One component of the force of eq. 2.17, -dphi + kappa rho dL + g, from dphi in PhiT.
// Near an interface close to equilibrium the two gradient terms almost cancel, so where
// phi is FP64 and the arithmetic FP32 the sum is formed in FP64 and rounded once (summed
// in FP32, its rounding moved a moving interface by ~3e-4 lattice units over 2000 steps,
// 8e-5 of the density).  Otherwise it is summed in the arithmetic type.  g64 is g in FP64.
template <class CD>
__device__ inline typename CD::C force_sum(PhiT<CD> gph, typename CD::C kappa, typename CD::C rh,
                                           typename CD::C gl, typename CD::C g, double g64) {
    using C = typename CD::C;
    if constexpr (!std::is_same<PhiT<CD>, C>::value)
        return C(-gph + double(kappa * rh * gl) + g64);
    else
        return -gph + kappa * rh * gl + g;
}

template <class C>
__device__ inline void grad3(const Row3<C>& s, const Row3<C>& m, const Row3<C>& n, C& gx, C& gy) {
    gx = C(1.0 / 3.0) * (m.e - m.w) + C(1.0 / 12.0) * ((n.e - n.w) + (s.e - s.w));
    gy = C(1.0 / 3.0) * (n.c - s.c) + C(1.0 / 12.0) * ((n.e + n.w) - (s.e + s.w));
}

// Wave-wide sum (64 lanes).
__device__ inline double wave_sum(double v) {
    // fixed butterfly: every lane ends with the same, order-deterministic sum
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Blocks are dispatched round-robin over the 8 XCDs of an MI355X; remap so that
// each XCD (own L2) works on a contiguous range of tiles, keeping the halo rows
// and columns that neighbouring strips share in one L2.
__device__ inline int xcd_remap(int b, int G) {
    const int xcd = b & 7, local = b >> 3, per = G >> 3, rem = G & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

// Pull-streaming of one node (column xe in [0, nx), row yr in [0, ny)).
// Populations whose source lies beyond a wall are bounced back (halfway
// bounce-back); sources beyond an end are clamped (extrapolated) or wrapped.
template <class CD>
__device__ inline void pull_generic(const typename CD::S* __restrict__ fin, const StepArgs& a, int xe, int yr,
                                    typename CD::C rho0, typename CD::C (&f)[9]) {
    using S = typename CD::S;
#define LBM_PULL(I)                                                                     \
    {                                                                                   \
        int sx = xe - ex(I), sy = yr - ey(I);                                           \
        const S* src;                                                                   \
        if (!a.yper && (sy < 0 || sy >= a.ny)) {                                        \
            src = fin + (long long)opp(I) * a.plane + (long long)yr * a.pitch + xe;     \
            f[I] = CD::template load<opp(I)>(src, rho0);                                \
        } else {                                                                        \
            if (a.yper) sy = wrapi(sy, a.ny);                                           \
            if (sx < 0 || sx >= a.nx) sx = a.xper ? wrapi(sx, a.nx) : clampi(sx, 0, a.nx - 1); \
            src = fin + (long long)(I) * a.plane + (long long)sy * a.pitch + sx;        \
            f[I] = CD::template load<I>(src, rho0);                                     \
        }                                                                               \
    }
    LBM_PULL(0) LBM_PULL(1) LBM_PULL(2) LBM_PULL(3) LBM_PULL(4) LBM_PULL(5) LBM_PULL(6) LBM_PULL(7) LBM_PULL(8)
#undef LBM_PULL
}

// Byte offset within a distribution buffer: 32-bit (the library keeps every
// buffer below 4 GiB), so loads and stores use a uniform 64-bit base in SGPRs
// plus one 32-bit lane offset (global_load v, v_off, s[base]).
template <class S>
__device__ inline const S* at_bytes(const S* base, uint32_t off) {
    return reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + (uint64_t)off);
}
template <class S>
__device__ inline S* at_bytes(S* base, uint32_t off) {
    return reinterpret_cast<S*>(reinterpret_cast<char*>(base) + (uint64_t)off);
}

// Raw buffer stores (a 128-bit resource in SGPRs, a 32-bit byte offset per
// lane).  The hardware range check drops a store whose offset is at or beyond
// the resource's size, so lanes that must not write are given kOobOffset
// instead of being masked off by a branch: the store sequence is then the same
// on every path, which keeps the compiler's load/store counter waits exact.
// Valid only while the buffer is smaller than 2 GiB, so that valid offsets stay
// below kOobOffset and kOobOffset plus any direction offset does not wrap.
constexpr uint32_t kOobOffset = 0x80000000u;
constexpr int kRawBufferWord3 = 0x00020000;  // 32-bit data format, no swizzle (gfx9 family)
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, kRawBufferWord3);
}
// soff is a uniform (SGPR) byte offset added to the lane offset off.
__device__ inline void buffer_store(double v, __amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, soff, 0);
}
__device__ inline void buffer_store(float v, __amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, soff, 0);
}
__device__ inline void buffer_store(_Float16 v, __amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, off, soff, 0);
}
__device__ inline void buffer_store(uint16_t v, __amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, off, soff, 0);
}
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ inline void buffer_store(Dual v, __amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, soff, 0);
}
template <class S>
__device__ inline S buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff);
template <>
__device__ inline Dual buffer_load<Dual>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_bit_cast(Dual, __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0));
}
template <>
__device__ inline double buffer_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
template <>
__device__ inline float buffer_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
template <>
__device__ inline _Float16 buffer_load<_Float16>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0));
}
template <>
__device__ inline uint16_t buffer_load<uint16_t>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0);
}

// Interior pull through a buffer resource: one lane offset per node and the
// nine uniform source offsets (direction plane minus the source displacement)
// in SGPRs, so the nine loads need no per-lane address arithmetic.
template <class CD>
__device__ inline void pull_interior_buf(__amdgpu_buffer_rsrc_t rin, const uint32_t (&dir_off)[9], uint32_t node_off,
                                         typename CD::C rho0, typename CD::C (&f)[9]) {
    using S = typename CD::S;
#define LBM_PULLB(I) f[I] = CD::template decode<I>(buffer_load<S>(rin, node_off, dir_off[I]), rho0);
    LBM_PULLB(0) LBM_PULLB(1) LBM_PULLB(2) LBM_PULLB(3) LBM_PULLB(4) LBM_PULLB(5) LBM_PULLB(6) LBM_PULLB(7) LBM_PULLB(8)
#undef LBM_PULLB
}

// Interior fast path: every source is in range, no boundary logic.  dir_off[I]
// is the uniform byte offset of population I's source relative to the node.
template <class CD>
__device__ inline void pull_interior(const typename CD::S* __restrict__ fin, const uint32_t (&dir_off)[9], uint32_t node_off,
                                     typename CD::C rho0, typename CD::C (&f)[9]) {
#define LBM_PULLI(I) f[I] = CD::template load<I>(at_bytes(fin, node_off + dir_off[I]), rho0);
    LBM_PULLI(0) LBM_PULLI(1) LBM_PULLI(2) LBM_PULLI(3) LBM_PULLI(4) LBM_PULLI(5) LBM_PULLI(6) LBM_PULLI(7) LBM_PULLI(8)
#undef LBM_PULLI
}

// MRT collision (eq. 2.1) in the Lallemand-Luo basis (rho, e, eps, jx, qx, jy, qy, pxx, pxy)
// with m_eq = M f_eq(rho, u_eq), eq. 2.2, and f* = f - M^-1 S (m - m_eq), M^-1 = M^T diag(1/|row|^2).
// f holds the working values (f itself, or the deviations f_i - k_i q of the shifted
// codecs), rho_m the density their energy moments pair with (moment_rho), inv_rho 1/rho.
template <class C>
__device__ inline void collide(C (&f)[9], C rho_m, C jx, C jy, C Fx, C Fy, C inv_rho, C tau, C s_e, C s_eps, C s_q,
                               C s_j, C s_v, C& vx, C& vy) {
    // P = rho u_eq = j + tau F exactly (velocity shift of Sec. 2.2); the reciprocal
    // of rho only enters the second-order terms, so mass and momentum updates do
    // not depend on its rounding.
    const C Px = jx + tau * Fx, Py = jy + tau * Fy;
    const C uex = Px * inv_rho, uey = Py * inv_rho;
    vx = (jx + C(0.5) * Fx) * inv_rho;
    vy = (jy + C(0.5) * Fy) * inv_rho;
    const C A = f[1] + f[2] + f[3] + f[4];
    const C D = f[5] + f[6] + f[7] + f[8];
    const C e = -C(4) * f[0] - A + C(2) * D;
    const C eps = C(4) * f[0] - C(2) * A + D;
    const C qx = C(2) * (f[3] - f[1]) + (f[5] - f[6] - f[7] + f[8]);
    const C qy = C(2) * (f[4] - f[2]) + (f[5] + f[6] - f[7] - f[8]);
    const C pxx = (f[1] + f[3]) - (f[2] + f[4]);
    const C pxy = (f[5] + f[7]) - (f[6] + f[8]);
    const C ru2 = C(3) * (Px * uex + Py * uey);  // 3 rho |u_eq|^2
    // relaxation terms d_k = S_k (m_k - m_eq_k) / |row_k|^2
    const C de = s_e * C(1.0 / 36.0) * (e - (ru2 - C(2) * rho_m));
    const C deps = s_eps * C(1.0 / 36.0) * (eps - (rho_m - ru2));
    const C djx = -s_j * tau * C(1.0 / 6.0) * Fx;
    const C djy = -s_j * tau * C(1.0 / 6.0) * Fy;
    const C dqx = s_q * C(1.0 / 12.0) * (qx + Px);
    const C dqy = s_q * C(1.0 / 12.0) * (qy + Py);
    const C dxx = s_v * C(0.25) * (pxx - (Px * uex - Py * uey));
    const C dxy = s_v * C(0.25) * (pxy - Px * uey);
    // f* = f - sum_k M_ki d_k
    const C c0 = -de - C(2) * deps;     // shared by the axis directions
    const C c1 = C(2) * de + deps;      // shared by the diagonals
    const C X = djx - C(2) * dqx, Y = djy - C(2) * dqy;
    const C Xd = djx + dqx, Yd = djy + dqy;
    f[0] -= C(4) * (deps - de);
    f[1] -= c0 + X + dxx;
    f[3] -= c0 - X + dxx;
    f[2] -= c0 + Y - dxx;
    f[4] -= c0 - Y - dxx;
    f[5] -= c1 + Xd + Yd + dxy;
    f[7] -= c1 - Xd - Yd + dxy;
    f[6] -= c1 - Xd + Yd - dxy;
    f[8] -= c1 + Xd - Yd - dxy;
}

// Loads (or, for rows beyond a wall, zeroes) the nine pulled populations of row r.
template <class CD>
__device__ inline void issue_row(const typename CD::S* __restrict__ fin, const StepArgs& a, int xe, bool strip_inner,
                                 const uint32_t (&dir_off)[9], int r, typename CD::C rho0, typename CD::C (&f)[9]) {
    using S = typename CD::S;
    if (a.yper || (r >= 0 && r < a.ny)) {
        const int yr = a.yper ? wrapi(r, a.ny) : r;
        if (strip_inner && yr >= 1 && yr <= a.ny - 2)
            pull_interior<CD>(fin, dir_off, uint32_t(yr * a.pitch + xe) * uint32_t(sizeof(S)), rho0, f);
        else
            pull_generic<CD>(fin, a, xe, yr, rho0, f);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = 0;
    }
}

// Per-wave register window of the row march.  Suffix 1 is row r-1, suffix 2
// row r-2 (the row being collided); lap3r is the Laplacian of row r-3.  P is the
// type of phi and its gradient.
template <class C, class P>
struct Window {
    Row3<C> rho1, rho2, lap2, lap3r;
    Row3<P> phi1, phi2;
    P gphx, gphy;             // grad phi of row r-2
    C grx, gry;               // grad rho of row r-2
    C f1[9], f2[9];           // pulled populations of rows r-1 and r-2
    C fn[9];                  // prefetched populations of row r
    C wall_rho, wall_vx, wall_p;
};

template <class CD, int EOS>
struct Stepper {
    using S = typename CD::S;
    using C = typename CD::C;
    const StepArgs& a;
    const S* __restrict__ fin;
    S* __restrict__ fout;
    int lane, strip, x, xe;
    bool out_lane, strip_inner;
    C rho0, RT, a_eff, bb, k2, kappa, g, tau, s_e, s_eps, s_q, s_j, s_v, rho_w, nu;
    uint32_t dir_off[9];  // byte offset of population i's pull source: i*plane - e_i (in elements) times sizeof(S)
    uint32_t plane_bytes;

    using P = PhiT<CD>;
    __device__ void prefetch(Window<C, P>& W, int r) const { issue_row<CD>(fin, a, xe, strip_inner, dir_off, r, rho0, W.fn); }

    // One row of the march: takes the prefetched populations of row r, issues
    // the loads of row r+1, forms rho/phi of row r and lap/grad of row r-1, and
    // (COLLIDE) updates row r-2.  WALL adds the wall-row logic; EMIT writes fields.
    // FAST: row r is a fluid row and row r+1 is an interior row of an interior
    // strip, so the prefetch is nine straight loads with no boundary logic.
    template <bool COLLIDE, bool WALL, bool EMIT, bool FAST>
    __device__ __forceinline__ void row(Window<C, P>& W, int r, bool prefetch_next) const {
        C f0[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) f0[i] = W.fn[i];
        if (FAST)
            pull_interior<CD>(fin, dir_off, uint32_t((r + 1) * a.pitch + xe) * uint32_t(sizeof(S)), rho0, W.fn);
        else if (prefetch_next)
            prefetch(W, r + 1);
        // Keep the loads of row r+1 ahead of this row's arithmetic and stores: on
        // gfx9 the vector-memory counter covers loads and stores in issue order, so
        // a load sunk below the stores would make its wait drain those stores too.
        __builtin_amdgcn_sched_barrier(0);
        const bool fluid_row = FAST || a.yper || (r >= 0 && r < a.ny);
        const C rho = fluid_row ? node_rho<CD>(f0, rho0) : rho_w;
        const Row3<C> rho0r = with_neighbours(rho);
        const Row3<P> phi0 = with_neighbours(phi_field<CD, EOS>(rho, a));
        const Row3<C> lap1 = with_neighbours(lap3(W.rho2, W.rho1, rho0r));
        P gphx1, gphy1;
        grad3(W.phi2, W.phi1, phi0, gphx1, gphy1);
        C grx1 = 0, gry1 = 0;
        if (WALL && !a.yper && (r - 1 == 0 || r - 1 == a.ny - 1)) grad3(W.rho2, W.rho1, rho0r, grx1, gry1);

        if (COLLIDE) {
            const int y = r - 2;
            C glx, gly;
            grad3(W.lap3r, W.lap2, lap1, glx, gly);
            const C rh = W.rho2.c;
            const C Fx = force_sum<CD>(W.gphx, kappa, rh, glx, g, a.g);
            const C Fy = force_sum<CD>(W.gphy, kappa, rh, gly, C(0), 0.0);
            C* f2 = W.f2;
            const C jx = (f2[1] - f2[3]) + (f2[5] - f2[6]) + (f2[8] - f2[7]);
            const C jy = (f2[2] - f2[4]) + (f2[5] - f2[8]) + (f2[6] - f2[7]);
            const C inv_rho = recip(rh);
            C vx, vy;
            collide<C>(W.f2, moment_rho<CD>(rh, rho0), jx, jy, Fx, Fy, inv_rho, tau, s_e, s_eps, s_q, s_j, s_v, vx, vy);
            if (out_lane) {
                const uint32_t o = uint32_t(y * a.pitch + x) * uint32_t(sizeof(S));
#define LBM_STORE(I) CD::template store<I>(at_bytes(fout, o + uint32_t(I) * plane_bytes), W.f2[I], rho0);
                LBM_STORE(0) LBM_STORE(1) LBM_STORE(2) LBM_STORE(3) LBM_STORE(4) LBM_STORE(5) LBM_STORE(6)
                LBM_STORE(7) LBM_STORE(8)
#undef LBM_STORE
                if (EMIT) {
                    const long long c = (long long)y * a.nx + x;
                    a.rho_out[c] = double(rh);
                    a.vx_out[c] = double(vx);
                    a.vy_out[c] = double(vy);
                }
            }
            if (WALL) wall_row(W, y, rh, vx);
        }
        // rotate the window
        W.rho2 = W.rho1; W.rho1 = rho0r;
        W.phi2 = W.phi1; W.phi1 = phi0;
        W.lap3r = W.lap2; W.lap2 = lap1;
        W.gphx = gphx1; W.gphy = gphy1;
        W.grx = grx1; W.gry = gry1;
#pragma unroll
        for (int i = 0; i < 9; ++i) { W.f2[i] = W.f1[i]; W.f1[i] = f0[i]; }
    }

    // Wall shear and wall pressure on the first two fluid rows of each wall
    // (FP64, into this step's slot of the wall ring).
    __device__ void wall_row(Window<C, P>& W, int y, C rh, C vx) const {
        if (a.yper) return;
        const bool bottom_p = (y == 0), top_p = (y == a.ny - 1);
        if (bottom_p || top_p) {
            // isotropic part of eq. 2.8 on the first fluid row
            W.wall_p = k2 * p0_of<EOS, C>(rh, RT, a_eff, bb) - kappa * rh * W.lap2.c
                     - C(0.5) * kappa * (W.grx * W.grx + W.gry * W.gry);
        }
        if (bottom_p) { W.wall_rho = rh; W.wall_vx = vx; }
        if (y == a.ny - 2) W.wall_vx = vx;
        const bool bottom_t = (y == 1), top_t = (y == a.ny - 1);
        if (!(bottom_t || top_t)) return;
        // tau_w = rho nu dv/ds, quadratic through v(0)=0, v(1/2), v(3/2)
        const C tw = bottom_t ? W.wall_rho * nu * (C(9) * W.wall_vx - vx) * C(1.0 / 3.0)
                              : rh * nu * (C(9) * vx - W.wall_vx) * C(1.0 / 3.0);
        const int w = bottom_t ? 0 : 1;
        if (out_lane) {
            a.tau_w[w * a.nx + x] = double(tw);
            a.p_w[w * a.nx + x] = double(W.wall_p);
            a.dtau_w[w * a.nx + x] = tangent_of(tw);
        }
    }
};

template <class CD, int EOS, bool EMIT>
__global__ __launch_bounds__(256) void step_kernel(const StepArgs a) {
    using C = typename CD::C;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int nbx = (a.nstrip + kWavesPerBlock - 1) / kWavesPerBlock;
    const int chunk = bid / nbx;
    const int strip = (bid - chunk * nbx) * kWavesPerBlock + wave;
    if (strip >= a.nstrip) return;  // whole wave

    Stepper<CD, EOS> st{a, static_cast<const typename CD::S*>(a.fin), static_cast<typename CD::S*>(a.fout)};
    st.lane = lane;
    st.strip = strip;
    const int x0 = strip * kStripOut;
    st.x = x0 - 2 + lane;
    st.out_lane = lane >= 2 && lane < 62 && st.x < a.nx;
    st.xe = st.x;
    if (st.xe < 0 || st.xe >= a.nx) st.xe = a.xper ? wrapi(st.xe, a.nx) : clampi(st.xe, 0, a.nx - 1);
    st.strip_inner = (x0 - 3 >= 0) && (x0 + 62 <= a.nx - 1);
    st.plane_bytes = uint32_t(a.plane) * uint32_t(sizeof(typename CD::S));
#pragma unroll
    for (int i = 0; i < 9; ++i)
        st.dir_off[i] = uint32_t(i) * st.plane_bytes - uint32_t(ey(i) * a.pitch + ex(i)) * uint32_t(sizeof(typename CD::S));
    st.rho0 = LBM_COEF(C, rho0); st.RT = LBM_COEF(C, RT); st.a_eff = LBM_COEF(C, a_eff);
    st.bb = LBM_COEF(C, b); st.k2 = LBM_COEF(C, k2); st.kappa = LBM_COEF(C, kappa); st.g = LBM_COEF(C, g);
    st.tau = LBM_COEF(C, tau); st.s_e = LBM_COEF(C, s_e); st.s_eps = LBM_COEF(C, s_eps); st.s_q = LBM_COEF(C, s_q);
    st.s_j = LBM_COEF(C, s_j); st.s_v = LBM_COEF(C, s_v); st.rho_w = LBM_COEF(C, rho_w); st.nu = LBM_COEF(C, nu);

    const int y0 = chunk * a.ty;
    const bool last = chunk == a.nchunk - 1;
    const int y1 = last ? a.ny : y0 + a.ty;
    const bool walls = !a.yper;
    // collided rows: [y0, y1).  The two wall-adjacent rows of the bottom (chunk 0)
    // and top (last chunk) go through the wall variant; the rest through the plain one.
    const int ya = (walls && chunk == 0) ? y0 + 2 : y0;
    const int yb = (walls && last) ? y1 - 2 : y1;

    Window<C, PhiT<CD>> W;
    W.rho1 = W.rho2 = W.lap2 = W.lap3r = Row3<C>{0, 0, 0};
    W.phi1 = W.phi2 = Row3<PhiT<CD>>{0, 0, 0};
    W.gphx = W.gphy = 0;
    W.grx = W.gry = 0;
    W.wall_rho = W.wall_vx = W.wall_p = 0;
#pragma unroll
    for (int i = 0; i < 9; ++i) { W.f1[i] = 0; W.f2[i] = 0; }

    const int rend = y1 + 2;  // rows y0-2 .. y1+1 are pulled
    st.prefetch(W, y0 - 2);
    // warm-up: rows y0-2 .. y0+1 only build the window (wall variant: grad rho of row 0)
    for (int r = y0 - 2; r < y0 + 2; ++r) st.template row<false, true, EMIT, false>(W, r, true);
    int r = y0 + 2;
    for (; r < ya + 2; ++r) st.template row<true, true, EMIT, false>(W, r, true);  // bottom wall rows
    if (st.strip_inner) {
        // interior rows whose prefetched row r+1 lies in 1 .. ny-2 (never true for y-periodic
        // wrap rows, which keep the generic path), three per trip: the window rotates with
        // period 3, so the rotation is register renaming in straight-line code
        const int rfast = a.yper ? r : (yb + 2 < a.ny - 2 ? yb + 2 : a.ny - 2);
        for (; r + 2 < rfast; r += 3) {
            st.template row<true, false, EMIT, true>(W, r, true);
            st.template row<true, false, EMIT, true>(W, r + 1, true);
            st.template row<true, false, EMIT, true>(W, r + 2, true);
        }
        for (; r < rfast; ++r) st.template row<true, false, EMIT, true>(W, r, true);
    }
    for (; r < yb + 2; ++r) st.template row<true, false, EMIT, false>(W, r, true);    // remaining interior rows
    for (; r < rend; ++r) st.template row<true, true, EMIT, false>(W, r, r + 1 < rend);  // top wall rows
}

// ---------------------------------------------------------------------------
// Tile schedule.  A block of 4 waves owns a 64-column x (TYO + 4)-row tile: the
// 60 output columns of a strip and TYO output rows, plus the radius-2 halo.
// Phase A: every thread pulls its rows (rows wave, wave + 4, ...: all loads of
//          a thread are independent and in flight together), forms rho and
//          phi and puts them in LDS; populations of output rows stay in registers.
// Phase B: Laplacian of rho on rows 1 .. H-2 of the tile, into LDS.
// Phase C: grad phi, grad lap, force, velocity shift, MRT collision, store.
// Phase D: (tiles holding a wall row) wall shear/pressure and per-strip extremes.
// Tiles are TYO rows apart; the last one is moved down to end at row ny - 1, so
// every tile has TYO output rows and the two rows next to a wall share a tile
// (rows covered by two tiles are computed identically by both).
// One tile of one lattice: `bid` is the tile index in tile-row-major order,
// fin/fout the distribution buffers of this step and tau_w/p_w/dtau_w its wall
// arrays (the kernels below pick them).  SAVE also writes the forward fields
// the adjoint of this step reads (a.save; layout of adjoint_field_elems).
// par is the step-counter parity of stochastic-rounding storage (unused otherwise).
template <class CD, int EOS, bool EMIT, int TYO, int NW, bool SAVE = false>
__device__ __forceinline__ void tile_body(const StepArgs& a, const void* fin_v, void* fout_v, double* tau_w,
                                          double* p_w, double* dtau_w, int bid, int par) {
    using S = typename CD::S;
    using C = typename CD::C;
    constexpr int H = TYO + 4;    // tile rows including the halo
    constexpr int RPT = H / NW;   // rows per thread
    static_assert(H % NW == 0, "tile height must be a multiple of the waves per block");
    using P = PhiT<CD>;
    __shared__ C sRho[H][64], sLap[H][64];
    __shared__ P sPhi[H][64];
    __shared__ C sWv[4][64], sWr[2][64], sWp[2][64];  // wall rows: vx (0, 1, ny-2, ny-1), rho and p_w (0, ny-1)

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // tile-row-major: consecutive blocks are x-neighbours, and with the XCD remap
    // each XCD walks a contiguous band of tile rows, so the halo columns and the
    // halo rows shared by neighbouring tiles are still in that XCD's L2
    const int tile = bid / a.nstrip;
    const int strip = bid - tile * a.nstrip;
    const int y0 = (a.ny >= TYO) ? min(tile * TYO, a.ny - TYO) : 0;
    const int x0 = strip * kStripOut;
    const int x = x0 - 2 + lane;
    const bool out_lane = lane >= 2 && lane < 62 && x < a.nx;
    int xe = x;
    if (xe < 0 || xe >= a.nx) xe = a.xper ? wrapi(xe, a.nx) : clampi(xe, 0, a.nx - 1);
    const bool strip_inner = (x0 - 3 >= 0) && (x0 + 62 <= a.nx - 1);
    const bool tile_inner = strip_inner && (y0 - 2 >= 1) && (y0 + H - 3 <= a.ny - 2);
    const bool walls = !a.yper;

    const S* __restrict__ fin = static_cast<const S*>(fin_v);
    S* __restrict__ fout = static_cast<S*>(fout_v);
    const uint32_t plane_bytes = uint32_t(a.plane) * uint32_t(sizeof(S));
    uint32_t dir_off[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) dir_off[i] = uint32_t(i) * plane_bytes - uint32_t(ey(i) * a.pitch + ex(i)) * uint32_t(sizeof(S));
    const C rho0 = LBM_COEF(C, rho0);
    const C RT = LBM_COEF(C, RT), a_eff = LBM_COEF(C, a_eff), bb = LBM_COEF(C, b);
    const C k2 = LBM_COEF(C, k2), kappa = LBM_COEF(C, kappa), g = LBM_COEF(C, g);
    const C rho_w = LBM_COEF(C, rho_w);
    // stochastic rounding: this step's counter seeds the random bits of every store;
    // one lane advances the counter of the next step (read by no block of this launch)
    uint32_t sr_seed = 0;
    if constexpr (stochastic_codec<CD>()) {
        const uint32_t step = a.sr[par];
        if (bid == 0 && threadIdx.x == 0) a.sr[1 - par] = step + 1u;
        sr_seed = hash32(step * 0x9e3779b9u + 0x632be5abu);
    }

    // ---- phase A: pull, density, EOS field -------------------------------------
    C f[RPT][9];
    if (tile_inner) {
        const __amdgpu_buffer_rsrc_t rin = buffer_rsrc(const_cast<S*>(fin), 9u * plane_bytes);
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int r = y0 - 2 + wave + NW * j;
            pull_interior_buf<CD>(rin, dir_off, uint32_t(r * a.pitch + xe) * uint32_t(sizeof(S)), rho0, f[j]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int r = y0 - 2 + wave + NW * j;
            if (a.yper || (r >= 0 && r < a.ny))
                pull_generic<CD>(fin, a, xe, a.yper ? wrapi(r, a.ny) : r, rho0, f[j]);
            else {
#pragma unroll
                for (int i = 0; i < 9; ++i) f[j][i] = 0;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int k = wave + NW * j;
        const int r = y0 - 2 + k;
        const bool fluid = tile_inner || a.yper || (r >= 0 && r < a.ny);
        const C rho = fluid ? node_rho<CD>(f[j], rho0) : rho_w;
        sRho[k][lane] = rho;
        sPhi[k][lane] = phi_field<CD, EOS>(rho, a);
    }
    __syncthreads();

    const int lm = lane > 0 ? lane - 1 : 0, lp = lane < 63 ? lane + 1 : 63;  // edge lanes are halo: clamped, unused
    // ---- phase B: Laplacian on rows 1 .. H-2 ------------------------------------
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int k = wave + NW * j;
        if (k >= 1 && k <= H - 2) {
            const Row3<C> s{sRho[k - 1][lane], sRho[k - 1][lp], sRho[k - 1][lm]};
            const Row3<C> m{sRho[k][lane], sRho[k][lp], sRho[k][lm]};
            const Row3<C> n{sRho[k + 1][lane], sRho[k + 1][lp], sRho[k + 1][lm]};
            sLap[k][lane] = lap3(s, m, n);
        }
    }
    __syncthreads();

    // ---- phase C: force, collision, store -----------------------------------------
    const bool wall_tile = walls && (y0 == 0 || y0 + TYO >= a.ny);
    const __amdgpu_buffer_rsrc_t rout = buffer_rsrc(fout, 9u * plane_bytes);
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int k = wave + NW * j;
        const int y = y0 - 2 + k;
        if (k < 2 || k > H - 3 || y >= a.ny) continue;  // halo row (wave-uniform)
        P gphx, gphy;
        C glx, gly;
        {
            const Row3<P> s{sPhi[k - 1][lane], sPhi[k - 1][lp], sPhi[k - 1][lm]};
            const Row3<P> m{sPhi[k][lane], sPhi[k][lp], sPhi[k][lm]};
            const Row3<P> n{sPhi[k + 1][lane], sPhi[k + 1][lp], sPhi[k + 1][lm]};
            grad3(s, m, n, gphx, gphy);
        }
        {
            const Row3<C> s{sLap[k - 1][lane], sLap[k - 1][lp], sLap[k - 1][lm]};
            const Row3<C> m{sLap[k][lane], sLap[k][lp], sLap[k][lm]};
            const Row3<C> n{sLap[k + 1][lane], sLap[k + 1][lp], sLap[k + 1][lm]};
            grad3(s, m, n, glx, gly);
        }
        const C rh = sRho[k][lane];
        const C Fx = force_sum<CD>(gphx, kappa, rh, glx, g, a.g);
        const C Fy = force_sum<CD>(gphy, kappa, rh, gly, C(0), 0.0);
        C* fj = f[j];
        const C jx = (fj[1] - fj[3]) + (fj[5] - fj[6]) + (fj[8] - fj[7]);
        const C jy = (fj[2] - fj[4]) + (fj[5] - fj[8]) + (fj[6] - fj[7]);
        C vx, vy;
        collide<C>(f[j], moment_rho<CD>(rh, rho0), jx, jy, Fx, Fy, recip(rh), LBM_COEF(C, tau), LBM_COEF(C, s_e),
                   LBM_COEF(C, s_eps), LBM_COEF(C, s_q), LBM_COEF(C, s_j), LBM_COEF(C, s_v), vx, vy);
        if (out_lane) {
            const uint32_t o = uint32_t(y * a.pitch + x) * uint32_t(sizeof(S));
            if constexpr (stochastic_codec<CD>()) {
                // 96 random bits per node and step: three hashes of (node, step), 10 bits of
                // its own per population in the top bits of its random word, so the nine
                // populations of a node round independently (words derived from one hash by
                // xorshift steps would carry only 32 bits of entropy per node).
                const uint32_t nd = uint32_t(y * a.pitch + x) * 3u;
                const uint32_t h[3] = {hash32(sr_seed ^ nd), hash32(sr_seed ^ (nd + 1u)), hash32(sr_seed ^ (nd + 2u))};
#define LBM_SSTORE(I) \
    buffer_store(CD::template encode_sr<I>(f[j][I], rho0, sr_word<I>(h)), rout, o, uint32_t(I) * plane_bytes);
                LBM_SSTORE(0) LBM_SSTORE(1) LBM_SSTORE(2) LBM_SSTORE(3) LBM_SSTORE(4) LBM_SSTORE(5) LBM_SSTORE(6)
                LBM_SSTORE(7) LBM_SSTORE(8)
#undef LBM_SSTORE
            } else {
#define LBM_TSTORE(I) buffer_store(CD::template encode<I>(f[j][I], rho0), rout, o, uint32_t(I) * plane_bytes);
                LBM_TSTORE(0) LBM_TSTORE(1) LBM_TSTORE(2) LBM_TSTORE(3) LBM_TSTORE(4) LBM_TSTORE(5) LBM_TSTORE(6)
                LBM_TSTORE(7) LBM_TSTORE(8)
#undef LBM_TSTORE
            }
            if (EMIT) {
                const long long c = (long long)y * a.nx + x;
                a.rho_out[c] = double(rh);
                a.vx_out[c] = double(vx);
                a.vy_out[c] = double(vy);
            }
            if (SAVE) {
                C* __restrict__ sv = static_cast<C*>(a.save);
                const long long o = (long long)y * a.pitch + x;
                const C inv = recip(rh), tau = LBM_COEF(C, tau);
                sv[o] = rh;
                sv[a.plane + o] = (jx + tau * Fx) * inv;
                sv[2 * a.plane + o] = (jy + tau * Fy) * inv;
                sv[3 * a.plane + o] = glx;
                sv[4 * a.plane + o] = gly;
                if (walls && (y <= 1 || y >= a.ny - 2)) {
                    const int w = y <= 1 ? y : 3 - (a.ny - 1 - y);
                    sv[5 * a.plane + (long long)w * a.nx + x] = vx;
                }
            }
        }
        if (wall_tile) {
            if (y == 0 || y == a.ny - 1) {
                // wall pressure: isotropic part of eq. 2.8 on the first fluid row
                const Row3<C> s{sRho[k - 1][lane], sRho[k - 1][lp], sRho[k - 1][lm]};
                const Row3<C> m{sRho[k][lane], sRho[k][lp], sRho[k][lm]};
                const Row3<C> n{sRho[k + 1][lane], sRho[k + 1][lp], sRho[k + 1][lm]};
                C grx, gry;
                grad3(s, m, n, grx, gry);
                const int w = (y == 0) ? 0 : 1;
                sWp[w][lane] = k2 * p0_of<EOS, C>(rh, RT, a_eff, bb) - kappa * rh * sLap[k][lane]
                             - C(0.5) * kappa * (grx * grx + gry * gry);
                sWr[w][lane] = rh;
            }
            if (y == 0) sWv[0][lane] = vx;
            if (y == 1) sWv[1][lane] = vx;
            if (y == a.ny - 2) sWv[2][lane] = vx;
            if (y == a.ny - 1) sWv[3][lane] = vx;
        }
    }

    // ---- phase D: wall shear and wall pressure into this step's wall arrays ----------
    if (!wall_tile) return;  // block-uniform
    __syncthreads();
    const bool has_bottom = (y0 == 0), has_top = (y0 + TYO >= a.ny);
    if ((wave == 0 && has_bottom) || (wave == 1 && has_top)) {
        const int w = wave;
        // tau_w = rho nu dv/ds, quadratic through v(0)=0, v(1/2), v(3/2)
        const C v_half = sWv[w == 0 ? 0 : 3][lane], v_3half = sWv[w == 0 ? 1 : 2][lane];
        const C tw = sWr[w][lane] * LBM_COEF(C, nu) * (C(9) * v_half - v_3half) * C(1.0 / 3.0);
        if (out_lane) {
            tau_w[w * a.nx + x] = double(tw);
            p_w[w * a.nx + x] = double(sWp[w][lane]);
            dtau_w[w * a.nx + x] = tangent_of(tw);
        }
    }
}

template <class CD, int EOS, bool EMIT, int TYO, int NW>
__global__ __launch_bounds__(64 * NW) void tile_kernel(const StepArgs a) {
    tile_body<CD, EOS, EMIT, TYO, NW>(a, a.fin, a.fout, a.tau_w, a.p_w, a.dtau_w, xcd_remap(blockIdx.x, gridDim.x),
                                      a.sr_par);
}

// Many lattices in one launch: the tiles of case c are blocks
// tile_start[c] .. tile_start[c+1]-1 (after the XCD remap).  The per-case
// arguments hold both distribution buffers (f[0] in fin, f[1] in fout) and the
// base of the wall ring; parity picks which buffer is read this step and slot
// the ring slot, the same for every case since the cases step together.
template <class CD, int EOS, bool EMIT, int TYO, int NW>
__global__ __launch_bounds__(64 * NW) void tile_batch_kernel(const StepArgs* __restrict__ cases,
                                                             const int* __restrict__ tile_start, int ncases,
                                                             int parity, int slot) {
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = ncases - 1;  // last case whose first tile is <= bid (uniform search)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= bid) lo = mid; else hi = mid - 1;
    }
    const StepArgs& a = cases[lo];
    const void* fin = parity ? a.fout : a.fin;
    void* fout = parity ? const_cast<void*>(a.fin) : a.fout;
    double* w = a.ring + (long long)slot * kWallSlotVals * a.nx;
    tile_body<CD, EOS, EMIT, TYO, NW>(a, fin, fout, w, w + 2 * a.nx, w + 4 * a.nx, bid - tile_start[lo], parity);
}

// ---------------------------------------------------------------------------
// Pipelined persistent tile schedule.  Same tiles and phases as tile_kernel,
// but each block stays resident and takes tile after tile, and the populations
// of its next tile are in flight while the current one is computed:
//
//   A(t)   rho, phi of tile t into LDS buffer (t's loads must have landed)
//   sync   the ticket of tile t+1 is visible; t+1's loads are issued
//   B(t)   Laplacian into LDS
//   sync
//   C(t)   force, collision and stores while t+1's loads are in flight
//   D(t)   wall tiles only
//
// rho and phi are double-buffered in LDS, so A(t+1) may start while slower
// waves still read tile t's values in C(t).  Wave w keeps output rows
// 2 + w + NW j (j < TYO / NW) in registers; waves 0..3 also pull one halo row
// each (rows 0, 1, H-2, H-1), which only feeds rho and phi.
//
// Tickets.  The tiles (row-major over strips) are cut into 8 contiguous ranges;
// blocks with blockIdx % 8 == g share counter g and walk range g, so with
// round-robin dispatch every XCD works through its own band of rows and keeps
// the shared halo rows in its L2.  Every block draws tickets until it draws one
// past the end of its range, so a launch consumes exactly (tiles of the range +
// blocks of the group) tickets and launch L of a run starts at L times that
// count; the host zeroes the counters before each run of launches.  A block
// draws the ticket of its tile after next while it computes, so the atomic's
// latency is hidden as well.  The order in which tiles are taken does not
// change any result: a tile reads only fin and writes only its own outputs.
template <class CD, int EOS, bool EMIT, int TYO, int NW>
struct Pipe {
    using S = typename CD::S;
    using C = typename CD::C;
    static constexpr int H = TYO + 4;                       // tile rows including the halo
    static constexpr int ORW = TYO / NW;                    // output rows per wave
    static constexpr int LRW = (TYO + 2 + NW - 1) / NW;     // Laplacian rows per wave
    static_assert(TYO % NW == 0 && NW >= 4, "tile rows must be a multiple of the waves, at least 4 waves");

    struct Smem {
        C rho[2][H][64], lap[H][64];
        PhiT<CD> phi[2][H][64];
        C wv[4][64], wr[2][64], wp[2][64];  // wall rows: vx (0, 1, ny-2, ny-1), rho and p_w (0, ny-1)
        int first, next;                    // broadcast tickets
    };

    struct Geom {
        int y0, x0, strip;
        bool inner, wall;
    };

    __device__ static Geom geom(const StepArgs& a, int t) {
        Geom g;
        const int tr = t / a.nstrip;
        g.strip = t - tr * a.nstrip;
        g.y0 = (a.ny >= TYO) ? min(tr * TYO, a.ny - TYO) : 0;
        g.x0 = g.strip * kStripOut;
        // every pulled source of the tile (rows y0-3 .. y0+TYO+2, columns x0-3 .. x0+62) is in range
        g.inner = (g.x0 - 3 >= 0) && (g.x0 + 62 <= a.nx - 1) && (g.y0 - 3 >= 0) && (g.y0 + TYO + 2 <= a.ny - 1);
        g.wall = !a.yper && (g.y0 == 0 || g.y0 + TYO >= a.ny);
        return g;
    }
    __device__ static int halo_k(int w) { return w < 2 ? w : H - 4 + w; }  // waves 0..3: rows 0, 1, H-2, H-1

    __device__ static int edge_x(const StepArgs& a, int x) {
        if (x < 0 || x >= a.nx) x = a.xper ? wrapi(x, a.nx) : clampi(x, 0, a.nx - 1);
        return x;
    }

    __device__ static void row_generic(const S* __restrict__ fin, const StepArgs& a, int xe, int r, C rho0, C (&f)[9]) {
        if (a.yper || (r >= 0 && r < a.ny)) {
            pull_generic<CD>(fin, a, xe, a.yper ? wrapi(r, a.ny) : r, rho0, f);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = 0;
        }
    }

    // Issues the loads of tile g's rows owned by wave w.
    __device__ static void issue(const S* __restrict__ fin, const StepArgs& a, const uint32_t (&dir_off)[9], const Geom& g,
                                 int w, int lane, C rho0, C (&fo)[ORW][9], C (&fh)[9]) {
        const int xe = edge_x(a, g.x0 - 2 + lane);
        if (g.inner) {
#pragma unroll
            for (int j = 0; j < ORW; ++j)
                pull_interior<CD>(fin, dir_off, uint32_t((g.y0 + w + NW * j) * a.pitch + xe) * uint32_t(sizeof(S)), rho0,
                                  fo[j]);
            if (w < 4)
                pull_interior<CD>(fin, dir_off, uint32_t((g.y0 - 2 + halo_k(w)) * a.pitch + xe) * uint32_t(sizeof(S)),
                                  rho0, fh);
        } else {
#pragma unroll
            for (int j = 0; j < ORW; ++j) row_generic(fin, a, xe, g.y0 + w + NW * j, rho0, fo[j]);
            if (w < 4) row_generic(fin, a, xe, g.y0 - 2 + halo_k(w), rho0, fh);
        }
    }

    __device__ static C density(const Geom& g, const StepArgs& a, int r, const C (&f)[9], C q, C rho_w) {
        const bool fluid = g.inner || a.yper || (r >= 0 && r < a.ny);
        return fluid ? node_rho<CD>(f, q) : rho_w;
    }

    // One tile: phases A-D on the populations fc (loaded earlier), issuing the
    // next tile's loads into fn.  Returns the next tile, or -1 when the range is done.
    template <int BUF>
    __device__ static int tile(Smem& sm, const StepArgs& a, const S* __restrict__ fin, S* __restrict__ fout,
                               const uint32_t (&dir_off)[9], int t, int t0, int nt, unsigned long long* ctr,
                               unsigned long long base, unsigned long long& tk, C (&fc)[ORW][9], C (&fn)[ORW][9],
                               C (&fh)[9]) {
        const int lane = threadIdx.x & 63;
        const int w = threadIdx.x >> 6;
        const Geom g = geom(a, t);
        const int x = g.x0 - 2 + lane;
        const bool out_lane = lane >= 2 && lane < 62 && x < a.nx;
        const C rho0 = LBM_COEF(C, rho0), rho_w = LBM_COEF(C, rho_w);
        const C RT = LBM_COEF(C, RT), a_eff = LBM_COEF(C, a_eff), bb = LBM_COEF(C, b);
        const C k2 = LBM_COEF(C, k2), kappa = LBM_COEF(C, kappa), gx = LBM_COEF(C, g);
        const int lm = lane > 0 ? lane - 1 : 0, lp = lane < 63 ? lane + 1 : 63;
        auto& sRho = sm.rho[BUF];
        auto& sPhi = sm.phi[BUF];
        const uint32_t plane_bytes = uint32_t(a.plane) * uint32_t(sizeof(S));
        const __amdgpu_buffer_rsrc_t rout = buffer_rsrc(fout, 9u * plane_bytes);

        // ---- A: density and EOS field of the owned rows -------------------------
#pragma unroll
        for (int j = 0; j < ORW; ++j) {
            const int k = 2 + w + NW * j;
            const C rho = density(g, a, g.y0 - 2 + k, fc[j], rho0, rho_w);
            sRho[k][lane] = rho;
            sPhi[k][lane] = phi_field<CD, EOS>(rho, a);
        }
        if (w < 4) {
            const int k = halo_k(w);
            const C rho = density(g, a, g.y0 - 2 + k, fh, rho0, rho_w);
            sRho[k][lane] = rho;
            sPhi[k][lane] = phi_field<CD, EOS>(rho, a);
        }
        if (threadIdx.x == 0) sm.next = int(tk - base);
        __syncthreads();

        // ---- next tile: its ticket is known, issue its loads ------------------------
        // unsigned: a ticket outside [0, nt) of any kind ends the block
        const int tn = __builtin_amdgcn_readfirstlane(sm.next);
        const bool more = unsigned(tn) < unsigned(nt);
        if (more) {
            if (threadIdx.x == 0) tk = atomicAdd(ctr, 1ull);  // ticket of the tile after next
            issue(fin, a, dir_off, geom(a, t0 + tn), w, lane, rho0, fn, fh);
        }

        // ---- B: Laplacian on rows 1 .. H-2 ---------------------------------------------
#pragma unroll
        for (int j = 0; j < LRW; ++j) {
            const int k = 1 + w + NW * j;
            if (k <= H - 2) {
                const Row3<C> s{sRho[k - 1][lane], sRho[k - 1][lp], sRho[k - 1][lm]};
                const Row3<C> m{sRho[k][lane], sRho[k][lp], sRho[k][lm]};
                const Row3<C> n{sRho[k + 1][lane], sRho[k + 1][lp], sRho[k + 1][lm]};
                sm.lap[k][lane] = lap3(s, m, n);
            }
        }
        __syncthreads();

        // ---- C: force, collision, store -------------------------------------------------
#pragma unroll
        for (int j = 0; j < ORW; ++j) {
            const int k = 2 + w + NW * j;
            const int y = g.y0 + w + NW * j;
            const bool row_ok = g.inner || y < a.ny;  // false only when ny < TYO (wave-uniform)
            PhiT<CD> gphx, gphy;
            C glx, gly;
            {
                const Row3<PhiT<CD>> s{sPhi[k - 1][lane], sPhi[k - 1][lp], sPhi[k - 1][lm]};
                const Row3<PhiT<CD>> m{sPhi[k][lane], sPhi[k][lp], sPhi[k][lm]};
                const Row3<PhiT<CD>> n{sPhi[k + 1][lane], sPhi[k + 1][lp], sPhi[k + 1][lm]};
                grad3(s, m, n, gphx, gphy);
            }
            {
                const Row3<C> s{sm.lap[k - 1][lane], sm.lap[k - 1][lp], sm.lap[k - 1][lm]};
                const Row3<C> m{sm.lap[k][lane], sm.lap[k][lp], sm.lap[k][lm]};
                const Row3<C> n{sm.lap[k + 1][lane], sm.lap[k + 1][lp], sm.lap[k + 1][lm]};
                grad3(s, m, n, glx, gly);
            }
            const C rh = sRho[k][lane];
            const C Fx = force_sum<CD>(gphx, kappa, rh, glx, gx, a.g);
            const C Fy = force_sum<CD>(gphy, kappa, rh, gly, C(0), 0.0);
            C* fj = fc[j];
            const C jx = (fj[1] - fj[3]) + (fj[5] - fj[6]) + (fj[8] - fj[7]);
            const C jy = (fj[2] - fj[4]) + (fj[5] - fj[8]) + (fj[6] - fj[7]);
            C vx, vy;
            collide<C>(fc[j], moment_rho<CD>(rh, rho0), jx, jy, Fx, Fy, recip(rh), LBM_COEF(C, tau), LBM_COEF(C, s_e), LBM_COEF(C, s_eps),
                       LBM_COEF(C, s_q), LBM_COEF(C, s_j), LBM_COEF(C, s_v), vx, vy);
            {
                const uint32_t o = (out_lane && row_ok) ? uint32_t(y * a.pitch + x) * uint32_t(sizeof(S)) : kOobOffset;
#define LBM_PSTORE(I) buffer_store(CD::template encode<I>(fc[j][I], rho0), rout, o + uint32_t(I) * plane_bytes);
                LBM_PSTORE(0) LBM_PSTORE(1) LBM_PSTORE(2) LBM_PSTORE(3) LBM_PSTORE(4) LBM_PSTORE(5) LBM_PSTORE(6)
                LBM_PSTORE(7) LBM_PSTORE(8)
#undef LBM_PSTORE
            }
            if (EMIT && out_lane && row_ok) {
                const long long c = (long long)y * a.nx + x;
                a.rho_out[c] = double(rh);
                a.vx_out[c] = double(vx);
                a.vy_out[c] = double(vy);
            }
            if (g.wall) {
                if (y == 0 || y == a.ny - 1) {
                    // wall pressure: isotropic part of eq. 2.8 on the first fluid row
                    const Row3<C> s{sRho[k - 1][lane], sRho[k - 1][lp], sRho[k - 1][lm]};
                    const Row3<C> m{sRho[k][lane], sRho[k][lp], sRho[k][lm]};
                    const Row3<C> n{sRho[k + 1][lane], sRho[k + 1][lp], sRho[k + 1][lm]};
                    C grx, gry;
                    grad3(s, m, n, grx, gry);
                    const int wi = (y == 0) ? 0 : 1;
                    sm.wp[wi][lane] = k2 * p0_of<EOS, C>(rh, RT, a_eff, bb) - kappa * rh * sm.lap[k][lane]
                                    - C(0.5) * kappa * (grx * grx + gry * gry);
                    sm.wr[wi][lane] = rh;
                }
                if (y == 0) sm.wv[0][lane] = vx;
                if (y == 1) sm.wv[1][lane] = vx;
                if (y == a.ny - 2) sm.wv[2][lane] = vx;
                if (y == a.ny - 1) sm.wv[3][lane] = vx;
            }
        }

        // ---- D: wall shear and wall pressure (wall tiles only) ----------------------------
        if (g.wall) {  // block-uniform
            __syncthreads();
            const bool has_bottom = (g.y0 == 0), has_top = (g.y0 + TYO >= a.ny);
            if ((w == 0 && has_bottom) || (w == 1 && has_top)) {
                // tau_w = rho nu dv/ds, quadratic through v(0)=0, v(1/2), v(3/2)
                const C v_half = sm.wv[w == 0 ? 0 : 3][lane], v_3half = sm.wv[w == 0 ? 1 : 2][lane];
                const C tw = sm.wr[w][lane] * LBM_COEF(C, nu) * (C(9) * v_half - v_3half) * C(1.0 / 3.0);
                if (out_lane) {
                    a.tau_w[w * a.nx + x] = double(tw);
                    a.p_w[w * a.nx + x] = double(sm.wp[w][lane]);
                    a.dtau_w[w * a.nx + x] = tangent_of(tw);
                }
            }
        }
        return more ? t0 + tn : -1;
    }
};

template <class CD, int EOS, bool EMIT, int TYO, int NW>
__global__ __launch_bounds__(64 * NW) void pipe_kernel(const StepArgs a) {
    using P = Pipe<CD, EOS, EMIT, TYO, NW>;
    using S = typename CD::S;
    using C = typename CD::C;
    __shared__ typename P::Smem sm;

    const int grp = blockIdx.x & 7;
    const int nb = (int(gridDim.x) - grp + 7) >> 3;  // blocks in this group
    const int ntiles = a.nstrip * ((a.ny + TYO - 1) / TYO);
    const int t0 = int(((long long)ntiles * grp) >> 3), t1 = int(((long long)ntiles * (grp + 1)) >> 3);
    const int nt = t1 - t0;
    unsigned long long* ctr = a.tickets + grp * kTicketStride;
    const unsigned long long base = (unsigned long long)a.launch * (unsigned long long)(nt + nb);

    if (threadIdx.x == 0) sm.first = int(atomicAdd(ctr, 1ull) - base);
    __syncthreads();
    const int first = __builtin_amdgcn_readfirstlane(sm.first);
    if (unsigned(first) >= unsigned(nt)) return;  // block-uniform: this block drew its one past-the-end ticket

    const S* __restrict__ fin = static_cast<const S*>(a.fin);
    S* __restrict__ fout = static_cast<S*>(a.fout);
    const uint32_t plane_bytes = uint32_t(a.plane) * uint32_t(sizeof(S));
    uint32_t dir_off[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) dir_off[i] = uint32_t(i) * plane_bytes - uint32_t(ey(i) * a.pitch + ex(i)) * uint32_t(sizeof(S));

    unsigned long long tk = 0;
    if (threadIdx.x == 0) tk = atomicAdd(ctr, 1ull);  // ticket of the second tile, before the first's loads
    C fa[P::ORW][9], fb[P::ORW][9], fh[9];
    int t = t0 + first;
    P::issue(fin, a, dir_off, P::geom(a, t), threadIdx.x >> 6, threadIdx.x & 63, LBM_COEF(C, rho0), fa, fh);
    for (;;) {
        t = P::template tile<0>(sm, a, fin, fout, dir_off, t, t0, nt, ctr, base, tk, fa, fb, fh);
        if (t < 0) break;
        t = P::template tile<1>(sm, a, fin, fout, dir_off, t, t0, nt, ctr, base, tk, fb, fa, fh);
        if (t < 0) break;
    }
}

// ---------------------------------------------------------------------------
// Two steps per launch (temporal blocking).  A block of NW waves owns a
// 64-column x (T + 10)-row tile: 54 output columns and T output rows plus a
// 5-node halo, which is what two steps need (a step reads the state within one
// node and the density within two more).  Step 1 runs from the state in global
// memory on the tile minus its outer 2 nodes and keeps its post-collision
// populations in LDS, encoded by the storage codec, so step 2 reads exactly
// the values a store and a reload would give.  Step 2 pulls them from LDS and
// collides the output nodes.  Every node is computed with tile_body's
// expressions, so one launch equals two one-step launches bit for bit while
// the state crosses HBM once per two steps.  Both steps write their wall
// arrays: step 1 to tau_w/p_w/dtau_w, step 2 to the next wall-ring slot
// (kWallSlotVals * nx further on).
constexpr int kHalo2 = 5;
static_assert(kStrip2Out + 2 * kHalo2 == 64, "a two-step tile is one wave wide");

template <class CD, int EOS, bool EMIT, int T, int NW>
__device__ __forceinline__ void tile2_body(const StepArgs& a, const void* fin_v, void* fout_v, double* tau_w,
                                           double* p_w, double* dtau_w, int bid) {
    using S = typename CD::S;
    using C = typename CD::C;
    constexpr int H = T + 2 * kHalo2;  // tile rows including the halo
    constexpr int H1 = H - 4;          // tile rows 2 .. H-3: step 1's collided nodes
    constexpr int RPT = H / NW;
    static_assert(H % NW == 0, "tile height must be a multiple of the waves per block");
    using P = PhiT<CD>;
    __shared__ C sRho[H][64], sLap[H][64];
    __shared__ P sPhi[H][64];
    __shared__ S sF[9][H1][64];
    __shared__ C sWv[2][4][64], sWr[2][2][64], sWp[2][2][64];  // wall rows of step 1 and step 2

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nstrip = (a.nx + kStrip2Out - 1) / kStrip2Out;
    const int tile = bid / nstrip;
    const int strip = bid - tile * nstrip;
    const int y0 = (a.ny >= T) ? min(tile * T, a.ny - T) : 0;
    const int x0 = strip * kStrip2Out;
    const int x = x0 - kHalo2 + lane;
    const bool xin = x >= 0 && x < a.nx;
    const bool xfl = a.xper || xin;  // a fluid column or a periodic image of one
    const bool out_lane = lane >= kHalo2 && lane < kHalo2 + kStrip2Out && x < a.nx;
    int xe = x;
    if (!xin) xe = a.xper ? wrapi(x, a.nx) : clampi(x, 0, a.nx - 1);
    // LDS lane of the node this lane stands for: itself, or for the copies beyond an
    // extrapolated end, the end column's lane
    const int lrep = xfl ? lane : xe - x0 + kHalo2;
    const bool tile_inner = (x0 - kHalo2 - 1 >= 0) && (x0 - kHalo2 + 64 <= a.nx - 1) && (y0 - kHalo2 - 1 >= 0) &&
                            (y0 + T + kHalo2 <= a.ny - 1);
    const bool walls = !a.yper;
    const bool wall_tile = walls && (y0 == 0 || y0 + T >= a.ny);  // block-uniform

    const S* __restrict__ fin = static_cast<const S*>(fin_v);
    S* __restrict__ fout = static_cast<S*>(fout_v);
    const uint32_t plane_bytes = uint32_t(a.plane) * uint32_t(sizeof(S));
    const C rho0 = LBM_COEF(C, rho0);
    const C RT = LBM_COEF(C, RT), a_eff = LBM_COEF(C, a_eff), bb = LBM_COEF(C, b);
    const C k2 = LBM_COEF(C, k2), kappa = LBM_COEF(C, kappa), g = LBM_COEF(C, g);
    const C rho_w = LBM_COEF(C, rho_w);
    const int lm = lane > 0 ? lane - 1 : 0, lp = lane < 63 ? lane + 1 : 63;  // edge lanes are halo: clamped, unused

    // Laplacian of sRho on this thread's tile rows klo .. khi
    auto laplacian = [&](int klo, int khi) {
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int k = wave + NW * j;
            if (k >= klo && k <= khi) {
                const Row3<C> s{sRho[k - 1][lane], sRho[k - 1][lp], sRho[k - 1][lm]};
                const Row3<C> m{sRho[k][lane], sRho[k][lp], sRho[k][lm]};
                const Row3<C> n{sRho[k + 1][lane], sRho[k + 1][lp], sRho[k + 1][lm]};
                sLap[k][lane] = lap3(s, m, n);
            }
        }
    };
    // Force and collision of the node at tile row k, pulled populations in fj (tile_body's
    // phase C); wall rows of output lanes record v_x, rho and p_w of step st.
    auto collide_at = [&](int k, int y, C (&fj)[9], int st, bool wall_lane, C& vx, C& vy) {
        P gphx, gphy;
        C glx, gly;
        {
            const Row3<P> s{sPhi[k - 1][lane], sPhi[k - 1][lp], sPhi[k - 1][lm]};
            const Row3<P> m{sPhi[k][lane], sPhi[k][lp], sPhi[k][lm]};
            const Row3<P> n{sPhi[k + 1][lane], sPhi[k + 1][lp], sPhi[k + 1][lm]};
            grad3(s, m, n, gphx, gphy);
        }
        {
            const Row3<C> s{sLap[k - 1][lane], sLap[k - 1][lp], sLap[k - 1][lm]};
            const Row3<C> m{sLap[k][lane], sLap[k][lp], sLap[k][lm]};
            const Row3<C> n{sLap[k + 1][lane], sLap[k + 1][lp], sLap[k + 1][lm]};
            grad3(s, m, n, glx, gly);
        }
        const C rh = sRho[k][lane];
        const C Fx = force_sum<CD>(gphx, kappa, rh, glx, g, a.g);
        const C Fy = force_sum<CD>(gphy, kappa, rh, gly, C(0), 0.0);
        const C jx = (fj[1] - fj[3]) + (fj[5] - fj[6]) + (fj[8] - fj[7]);
        const C jy = (fj[2] - fj[4]) + (fj[5] - fj[8]) + (fj[6] - fj[7]);
        collide<C>(fj, moment_rho<CD>(rh, rho0), jx, jy, Fx, Fy, recip(rh), LBM_COEF(C, tau), LBM_COEF(C, s_e), LBM_COEF(C, s_eps),
                   LBM_COEF(C, s_q), LBM_COEF(C, s_j), LBM_COEF(C, s_v), vx, vy);
        if (wall_lane) {
            if (y == 0 || y == a.ny - 1) {
                // wall pressure: isotropic part of eq. 2.8 on the first fluid row
                const Row3<C> s{sRho[k - 1][lane], sRho[k - 1][lp], sRho[k - 1][lm]};
                const Row3<C> m{sRho[k][lane], sRho[k][lp], sRho[k][lm]};
                const Row3<C> n{sRho[k + 1][lane], sRho[k + 1][lp], sRho[k + 1][lm]};
                C grx, gry;
                grad3(s, m, n, grx, gry);
                const int w = (y == 0) ? 0 : 1;
                sWp[st][w][lane] = k2 * p0_of<EOS, C>(rh, RT, a_eff, bb) - kappa * rh * sLap[k][lane]
                                 - C(0.5) * kappa * (grx * grx + gry * gry);
                sWr[st][w][lane] = rh;
            }
            if (y == 0) sWv[st][0][lane] = vx;
            if (y == 1) sWv[st][1][lane] = vx;
            if (y == a.ny - 2) sWv[st][2][lane] = vx;
            if (y == a.ny - 1) sWv[st][3][lane] = vx;
        }
    };
    // Wall shear of step st from the recorded rows (waves 0 and 1; tile_body's phase D).
    auto wall_shear = [&](int st, double* tw_out, double* pw_out, double* dtw_out) {
        const bool has_bottom = (y0 == 0), has_top = (y0 + T >= a.ny);
        if ((wave == 0 && has_bottom) || (wave == 1 && has_top)) {
            const int w = wave;
            // tau_w = rho nu dv/ds, quadratic through v(0)=0, v(1/2), v(3/2)
            const C v_half = sWv[st][w == 0 ? 0 : 3][lane], v_3half = sWv[st][w == 0 ? 1 : 2][lane];
            const C tw = sWr[st][w][lane] * LBM_COEF(C, nu) * (C(9) * v_half - v_3half) * C(1.0 / 3.0);
            if (out_lane) {
                tw_out[w * a.nx + x] = double(tw);
                pw_out[w * a.nx + x] = double(sWp[st][w][lane]);
                dtw_out[w * a.nx + x] = tangent_of(tw);
            }
        }
    };
    auto density = [&](const C (&f)[9]) { return node_rho<CD>(f, rho0); };

    // ---- step 1, phase A: pull from global memory, density, EOS field on all rows ------
    {
        C f[RPT][9];
        if (tile_inner) {
            uint32_t dir_off[9];
#pragma unroll
            for (int i = 0; i < 9; ++i)
                dir_off[i] = uint32_t(i) * plane_bytes - uint32_t(ey(i) * a.pitch + ex(i)) * uint32_t(sizeof(S));
            const __amdgpu_buffer_rsrc_t rin = buffer_rsrc(const_cast<S*>(fin), 9u * plane_bytes);
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int r = y0 - kHalo2 + wave + NW * j;
                pull_interior_buf<CD>(rin, dir_off, uint32_t(r * a.pitch + xe) * uint32_t(sizeof(S)), rho0, f[j]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int r = y0 - kHalo2 + wave + NW * j;
                if (a.yper || (r >= 0 && r < a.ny))
                    pull_generic<CD>(fin, a, xe, a.yper ? wrapi(r, a.ny) : r, rho0, f[j]);
                else {
#pragma unroll
                    for (int i = 0; i < 9; ++i) f[j][i] = 0;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int k = wave + NW * j;
            const int r = y0 - kHalo2 + k;
            const bool fluid = tile_inner || a.yper || (r >= 0 && r < a.ny);
            const C rho = fluid ? density(f[j]) : rho_w;
            sRho[k][lane] = rho;
            sPhi[k][lane] = phi_field<CD, EOS>(rho, a);
        }
        __syncthreads();
        // ---- step 1, phase B: Laplacian on rows 1 .. H-2 -------------------------------
        laplacian(1, H - 2);
        __syncthreads();
        // ---- step 1, phase C: collide rows 2 .. H-3 and keep them (encoded) in LDS -----
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int k = wave + NW * j;
            const int y = y0 - kHalo2 + k;
            if (k < 2 || k > H - 3) continue;                          // wave-uniform
            if (!(a.yper || (y >= 0 && y < a.ny)) || !xfl) continue;   // ghost rows and end copies: never read
            C vx, vy;
            const bool wall_lane = wall_tile && out_lane && k >= kHalo2 && k < kHalo2 + T;
            collide_at(k, y, f[j], 0, wall_lane, vx, vy);
#define LBM_KEEP(I) sF[I][k - 2][lane] = CD::template encode<I>(f[j][I], rho0);
            LBM_KEEP(0) LBM_KEEP(1) LBM_KEEP(2) LBM_KEEP(3) LBM_KEEP(4) LBM_KEEP(5) LBM_KEEP(6) LBM_KEEP(7) LBM_KEEP(8)
#undef LBM_KEEP
        }
    }
    __syncthreads();
    if (wall_tile) wall_shear(0, tau_w, p_w, dtau_w);

    // ---- step 2, phase A: pull from LDS on rows 3 .. H-4 (lanes 3 .. 60), density, EOS ---
    // Sources follow the one-step pull: beyond a wall the node's own opposite
    // population, beyond an extrapolated end the end column, periodic images by lane.
    C f2[RPT][9];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int k = wave + NW * j;
        const int r = y0 - kHalo2 + k;
#pragma unroll
        for (int i = 0; i < 9; ++i) f2[j][i] = 0;
        if (k < 3 || k > H - 4) continue;  // wave-uniform
        const bool fluid = a.yper || (r >= 0 && r < a.ny);
        if (fluid && lane >= 3 && lane <= 60) {
            const int yr = a.yper ? wrapi(r, a.ny) : r;
#define LBM_PULL2(I)                                                                                          \
    {                                                                                                         \
        const int sy = yr - ey(I);                                                                            \
        if (tile_inner) {                                                                                     \
            f2[j][I] = CD::template decode<I>(sF[I][k - ey(I) - 2][lane - ex(I)], rho0);                      \
        } else if (!a.yper && (sy < 0 || sy >= a.ny)) {                                                       \
            f2[j][I] = CD::template decode<opp(I)>(sF[opp(I)][k - 2][lrep], rho0);                            \
        } else {                                                                                              \
            const int sx = xe - ex(I);                                                                        \
            const int ls = (a.xper || (sx >= 0 && sx < a.nx)) ? lrep - ex(I) : clampi(sx, 0, a.nx - 1) - x0 + kHalo2; \
            f2[j][I] = CD::template decode<I>(sF[I][k - ey(I) - 2][ls], rho0);                                \
        }                                                                                                     \
    }
            LBM_PULL2(0) LBM_PULL2(1) LBM_PULL2(2) LBM_PULL2(3) LBM_PULL2(4) LBM_PULL2(5) LBM_PULL2(6) LBM_PULL2(7)
            LBM_PULL2(8)
#undef LBM_PULL2
        }
        const C rho = fluid ? density(f2[j]) : rho_w;
        sRho[k][lane] = rho;
        sPhi[k][lane] = phi_field<CD, EOS>(rho, a);
    }
    __syncthreads();
    // ---- step 2, phase B: Laplacian on rows 4 .. H-5 -------------------------------------
    laplacian(4, H - 5);
    __syncthreads();
    // ---- step 2, phase C: collide the output rows, store ---------------------------------
    const __amdgpu_buffer_rsrc_t rout = buffer_rsrc(fout, 9u * plane_bytes);
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int k = wave + NW * j;
        const int y = y0 - kHalo2 + k;
        if (k < kHalo2 || k >= kHalo2 + T || y >= a.ny) continue;  // wave-uniform
        C vx, vy;
        collide_at(k, y, f2[j], 1, wall_tile && out_lane, vx, vy);
        if (out_lane) {
            const uint32_t o = uint32_t(y * a.pitch + x) * uint32_t(sizeof(S));
#define LBM_TSTORE(I) buffer_store(CD::template encode<I>(f2[j][I], rho0), rout, o, uint32_t(I) * plane_bytes);
            LBM_TSTORE(0) LBM_TSTORE(1) LBM_TSTORE(2) LBM_TSTORE(3) LBM_TSTORE(4) LBM_TSTORE(5) LBM_TSTORE(6)
            LBM_TSTORE(7) LBM_TSTORE(8)
#undef LBM_TSTORE
            if (EMIT) {
                const long long c = (long long)y * a.nx + x;
                a.rho_out[c] = double(sRho[k][lane]);
                a.vx_out[c] = double(vx);
                a.vy_out[c] = double(vy);
            }
        }
    }
    if (!wall_tile) return;  // block-uniform
    __syncthreads();
    const long long next = (long long)kWallSlotVals * a.nx;
    wall_shear(1, tau_w + next, p_w + next, dtau_w + next);
}

template <class CD, int EOS, bool EMIT, int T, int NW>
__global__ __launch_bounds__(64 * NW) void tile2_kernel(const StepArgs a) {
    tile2_body<CD, EOS, EMIT, T, NW>(a, a.fin, a.fout, a.tau_w, a.p_w, a.dtau_w, xcd_remap(blockIdx.x, gridDim.x));
}

// Two steps of many lattices in one launch: tile_batch_kernel's layout with the
// two-step tiles (tile_start counts them), the two steps' wall arrays in ring
// slots slot and slot + 1.
template <class CD, int EOS, bool EMIT, int T, int NW>
__global__ __launch_bounds__(64 * NW) void tile2_batch_kernel(const StepArgs* __restrict__ cases,
                                                              const int* __restrict__ tile_start, int ncases,
                                                              int parity, int slot) {
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    int lo = 0, hi = ncases - 1;  // last case whose first tile is <= bid (uniform search)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile_start[mid] <= bid) lo = mid; else hi = mid - 1;
    }
    const StepArgs& a = cases[lo];
    const void* fin = parity ? a.fout : a.fin;
    void* fout = parity ? const_cast<void*>(a.fin) : a.fout;
    double* w = a.ring + (long long)slot * kWallSlotVals * a.nx;
    tile2_body<CD, EOS, EMIT, T, NW>(a, fin, fout, w, w + 2 * a.nx, w + 4 * a.nx, bid - tile_start[lo]);
}

template <class CD, int EOS, int TYO, int NW>
hipError_t launch_tile(const StepArgs& a, bool emit, hipStream_t s) {
    const dim3 grid(a.nstrip * ((a.ny + TYO - 1) / TYO)), block(64 * NW);
    if (emit)
        hipLaunchKernelGGL((tile_kernel<CD, EOS, true, TYO, NW>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((tile_kernel<CD, EOS, false, TYO, NW>), grid, block, 0, s, a);
    return hipGetLastError();
}

// Two steps in one launch (tile2_kernel) over 54-column strips.
template <class CD, int EOS, int T, int NW>
hipError_t launch_tile2(const StepArgs& a, bool emit, hipStream_t s) {
    const dim3 grid(tiles2(a.nx, a.ny, T)), block(64 * NW);
    if (emit)
        hipLaunchKernelGGL((tile2_kernel<CD, EOS, true, T, NW>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((tile2_kernel<CD, EOS, false, T, NW>), grid, block, 0, s, a);
    return hipGetLastError();
}

// Tile of the two-step kernel: 14 output rows and 8 waves with FP32 arithmetic,
// 6 rows and 4 waves with FP64 arithmetic (LDS holds a step of populations).
template <class CD>
hipError_t launch_step2_c(const StepArgs& a, int eos, bool emit, hipStream_t s) {
    constexpr bool f64 = sizeof(typename CD::C) == 8;
    constexpr int T = f64 ? 6 : 14, NW = f64 ? 4 : 8;
    static_assert(T == (f64 ? kTile2RowsF64 : kTile2Rows), "two-step tile rows");
    return eos == LBM_EOS_CS ? launch_tile2<CD, LBM_EOS_CS, T, NW>(a, emit, s) : launch_tile2<CD, LBM_EOS_PR, T, NW>(a, emit, s);
}

template <class CD, int EOS>
hipError_t launch_batch2_e(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, int parity,
                           int slot, bool emit, hipStream_t s) {
    constexpr bool f64 = sizeof(typename CD::C) == 8;
    constexpr int T = f64 ? 6 : 14, NW = f64 ? 4 : 8;
    const dim3 grid(total_tiles), block(64 * NW);
    if (emit)
        hipLaunchKernelGGL((tile2_batch_kernel<CD, EOS, true, T, NW>), grid, block, 0, s, cases, tile_start, ncases,
                           parity, slot);
    else
        hipLaunchKernelGGL((tile2_batch_kernel<CD, EOS, false, T, NW>), grid, block, 0, s, cases, tile_start, ncases,
                           parity, slot);
    return hipGetLastError();
}
template <class CD>
hipError_t launch_batch2_c(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, int parity,
                           int slot, int eos, bool emit, hipStream_t s) {
    return eos == LBM_EOS_CS ? launch_batch2_e<CD, LBM_EOS_CS>(cases, tile_start, ncases, total_tiles, parity, slot, emit, s)
                             : launch_batch2_e<CD, LBM_EOS_PR>(cases, tile_start, ncases, total_tiles, parity, slot, emit, s);
}

template <class CD, int EOS, int TYO, int NW>
hipError_t launch_batch_t(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, int parity,
                          int slot, bool emit, hipStream_t s) {
    const dim3 grid(total_tiles), block(64 * NW);
    if (emit)
        hipLaunchKernelGGL((tile_batch_kernel<CD, EOS, true, TYO, NW>), grid, block, 0, s, cases, tile_start, ncases,
                           parity, slot);
    else
        hipLaunchKernelGGL((tile_batch_kernel<CD, EOS, false, TYO, NW>), grid, block, 0, s, cases, tile_start, ncases,
                           parity, slot);
    return hipGetLastError();
}

template <class CD, int EOS>
hipError_t launch_batch_e(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, int parity,
                          int slot, int ty, int waves, bool emit, hipStream_t s) {
    if (waves == 8) {
        switch (ty) {
            case 12: return launch_batch_t<CD, EOS, 12, 8>(cases, tile_start, ncases, total_tiles, parity, slot, emit, s);
            case 20: return launch_batch_t<CD, EOS, 20, 8>(cases, tile_start, ncases, total_tiles, parity, slot, emit, s);
            case 28: return launch_batch_t<CD, EOS, 28, 8>(cases, tile_start, ncases, total_tiles, parity, slot, emit, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (ty) {
        case 8: return launch_batch_t<CD, EOS, 8, 4>(cases, tile_start, ncases, total_tiles, parity, slot, emit, s);
        case 12: return launch_batch_t<CD, EOS, 12, 4>(cases, tile_start, ncases, total_tiles, parity, slot, emit, s);
        case 20: return launch_batch_t<CD, EOS, 20, 4>(cases, tile_start, ncases, total_tiles, parity, slot, emit, s);
        case 28: return launch_batch_t<CD, EOS, 28, 4>(cases, tile_start, ncases, total_tiles, parity, slot, emit, s);
        default: return hipErrorInvalidValue;
    }
}

template <class CD>
hipError_t launch_batch_c(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, int parity,
                          int slot, int eos, int ty, int waves, bool emit, hipStream_t s) {
    return eos == LBM_EOS_CS
               ? launch_batch_e<CD, LBM_EOS_CS>(cases, tile_start, ncases, total_tiles, parity, slot, ty, waves, emit, s)
               : launch_batch_e<CD, LBM_EOS_PR>(cases, tile_start, ncases, total_tiles, parity, slot, ty, waves, emit, s);
}

template <class CD, int EOS, int TYO, int NW>
hipError_t launch_pipe(const StepArgs& a, bool emit, hipStream_t s) {
    const dim3 grid(a.pipe_blocks), block(64 * NW);
    if (emit)
        hipLaunchKernelGGL((pipe_kernel<CD, EOS, true, TYO, NW>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((pipe_kernel<CD, EOS, false, TYO, NW>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <class CD, int EOS>
hipError_t launch_step_t(const StepArgs& a, bool emit, hipStream_t s) {
    if (a.schedule == kSchedulePipe) {
        if (a.tile_waves == 8) {
            switch (a.ty) {
                case 8: return launch_pipe<CD, EOS, 8, 8>(a, emit, s);
                case 16: return launch_pipe<CD, EOS, 16, 8>(a, emit, s);
                default: return hipErrorInvalidValue;
            }
        }
        switch (a.ty) {
            case 4: return launch_pipe<CD, EOS, 4, 4>(a, emit, s);
            case 8: return launch_pipe<CD, EOS, 8, 4>(a, emit, s);
            case 12: return launch_pipe<CD, EOS, 12, 4>(a, emit, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (a.schedule == kScheduleTile) {
        if (a.tile_waves == 8) {
            switch (a.ty) {
                case 12: return launch_tile<CD, EOS, 12, 8>(a, emit, s);
                case 20: return launch_tile<CD, EOS, 20, 8>(a, emit, s);
                case 28: return launch_tile<CD, EOS, 28, 8>(a, emit, s);
                default: return hipErrorInvalidValue;
            }
        }
        switch (a.ty) {
            case 8: return launch_tile<CD, EOS, 8, 4>(a, emit, s);
            case 12: return launch_tile<CD, EOS, 12, 4>(a, emit, s);
            case 20: return launch_tile<CD, EOS, 20, 4>(a, emit, s);
            case 28: return launch_tile<CD, EOS, 28, 4>(a, emit, s);
            default: return hipErrorInvalidValue;
        }
    }
    const int nbx = (a.nstrip + kWavesPerBlock - 1) / kWavesPerBlock;
    const dim3 grid(nbx * a.nchunk), block(64 * kWavesPerBlock);
    if (emit)
        hipLaunchKernelGGL((step_kernel<CD, EOS, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((step_kernel<CD, EOS, false>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <class CD>
hipError_t launch_step_c(const StepArgs& a, int eos, bool emit, hipStream_t s) {
    return eos == LBM_EOS_CS ? launch_step_t<CD, LBM_EOS_CS>(a, emit, s) : launch_step_t<CD, LBM_EOS_PR>(a, emit, s);
}


template <class CD, int EOS>
hipError_t pipe_grid_t(int ty, int waves, int* blocks) {
    const void* k = nullptr;
#define LBM_PK(T, W) reinterpret_cast<const void*>(&pipe_kernel<CD, EOS, false, T, W>)
    if (waves == 8) k = ty == 8 ? LBM_PK(8, 8) : ty == 16 ? LBM_PK(16, 8) : nullptr;
    else k = ty == 4 ? LBM_PK(4, 4) : ty == 8 ? LBM_PK(8, 4) : ty == 12 ? LBM_PK(12, 4) : nullptr;
#undef LBM_PK
    if (!k) return hipErrorInvalidValue;
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, 64 * waves, 0);
    if (e != hipSuccess) return e;
    *blocks = (cus > 0 ? cus : 1) * (per > 0 ? per : 1);
    return hipSuccess;
}
template <class CD>
hipError_t pipe_grid_c(int eos, int ty, int waves, int* blocks) {
    return eos == LBM_EOS_CS ? pipe_grid_t<CD, LBM_EOS_CS>(ty, waves, blocks) : pipe_grid_t<CD, LBM_EOS_PR>(ty, waves, blocks);
}

}  // namespace
}  // namespace lbm

// Defines the exported launchers of one storage type (one translation unit each).
#define LBM_DEFINE_STORAGE_LAUNCHERS(NAME, CODEC)                                                              \
    namespace lbm {                                                                                            \
    hipError_t launch_step_##NAME(const StepArgs& a, int eos, bool emit, hipStream_t s) {                     \
        return launch_step_c<CODEC>(a, eos, emit, s);                                                          \
    }                                                                                                          \
    hipError_t launch_batch_##NAME(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles,  \
                                   int parity, int slot, int eos, int ty, int waves, bool emit, hipStream_t s) { \
        return launch_batch_c<CODEC>(cases, tile_start, ncases, total_tiles, parity, slot, eos, ty, waves, emit, s); \
    }                                                                                                          \
    hipError_t pipe_grid_##NAME(int eos, int ty, int waves, int* blocks) {                                     \
        return pipe_grid_c<CODEC>(eos, ty, waves, blocks);                                                     \
    }                                                                                                          \
    hipError_t launch_step2_##NAME(const StepArgs& a, int eos, bool emit, hipStream_t s) {                    \
        return launch_step2_c<CODEC>(a, eos, emit, s);                                                         \
    }                                                                                                          \
    hipError_t launch_batch2_##NAME(const StepArgs* cases, const int* tile_start, int ncases, int total_tiles, \
                                    int parity, int slot, int eos, bool emit, hipStream_t s) {                \
        return launch_batch2_c<CODEC>(cases, tile_start, ncases, total_tiles, parity, slot, eos, emit, s);     \
    }                                                                                                          \
    }
