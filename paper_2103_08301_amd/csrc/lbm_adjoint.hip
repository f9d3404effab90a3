// lbm_adjoint.hip -- reverse-mode (adjoint) step of the EOS-based multiphase
// MRT lattice Boltzmann method (arXiv 2103.08301, Sec. 2).
//
// Objective: J = sum over steps, walls and columns of tau_w^2 (the time
// integral of the squared wall shear of Figs. 3, 5 and 8).  One launch takes
// the adjoint of one step n backwards: given lam_in = dJ/df(x) of step n + 1's
// pulled populations (before its own streaming adjoint), it produces lam_out,
// the same quantity for step n, and the step's contribution to dJ/dtheta.
//
// Forward step n, per fluid node (eqs. 2.1, 2.2, 2.12, 2.17; Sec. 2.2-2.3):
//   f_i(x)  = f*_{i}(x - e_i)            (bounce-back / clamped / wrapped)
//   rho, j  = sum f_i, sum e_i f_i
//   phi     = k^2 p0(rho) - rho/3,  L = lap rho,  F = -grad phi + kappa rho grad L + (g, 0)
//   P       = j + tau F,  u = P / rho,  v = (j + F/2) / rho
//   f*      = f - M^-1 S (M f - m_eq(rho, P))
//   tau_w   = rho nu (9 v_x(s=1/2) - v_x(s=3/2)) / 3 on the two rows next to a wall
// The adjoint runs these in reverse with the transposed operators: the
// collision's Jacobian in f is the constant symmetric I - M^T D M (D = S /
// |row|^2), the gradient stencil transposes to minus a divergence and the
// Laplacian to itself, ghost copies of the end columns add their adjoints back
// into the copied column, and the pull transposes to a gather of lam_in from
// the downstream neighbours x + e_i (bounce-back from the node itself).
//
// The backward sweep recomputes each checkpoint segment forwards with a step
// kernel that also writes the forward quantities this adjoint needs (rho, u =
// (j + tau F)/rho, grad lap rho, and v_x on the wall rows), so the adjoint
// recomputes none of the step.  A tile of 64 columns (60 outputs and a 2-column
// halo on each side) by TYO + 4 rows: the force adjoint is needed within 1 node
// of the outputs' density adjoint and within 2 nodes of the outputs, and at a
// node it depends only on lam and that node's forward fields.  Phases, with
// barriers between them:
//   A  gather lam, the collision's vector-Jacobian product: the local part of
//      dJ/df (output rows) and the force adjoint F~ (all rows), rho and F~ to LDS
//   D  phi~ = div F~ and L~ = -div(kappa rho F~) (radius 1)
//   E  rho~ = lap L~ + phi'(rho) phi~ (+ ghost columns), store dJ/df, and the
//      parameter sums sum F~_x, sum phi~ dphi/d(RT, a_eff, b)
// No MFMA: like the forward step this is a bandwidth-bound stencil.
#include "lbm_device.hpp"

namespace lbm {
namespace {

constexpr int kAdjHalo = 2;

// dphi/drho and dphi/d(RT, a_eff, b) of phi = k^2 p0(rho) - rho/3 at one density
// (the same p0 as phi_of: eq. A9 with the van der Waals attraction, eq. A8).
template <int EOS, class C>
__device__ inline void phi_partials(C rho, C RT, C a_eff, C b, C k2, C& d_rho, C& d_RT, C& d_a, C& d_b) {
    if (EOS == LBM_EOS_CS) {
        // p0 = rho RT Z(eta) - a rho^2, Z = (1 + eta + eta^2 - eta^3)/(1 - eta)^3, eta = b rho/4
        const C eta = C(0.25) * b * rho;
        const C num = C(1) + eta * (C(1) + eta * (C(1) - eta));
        const C dnum = C(1) + eta * (C(2) - C(3) * eta);
        const C d = C(1) - eta;
        const C id = recip(d);
        const C id3 = id * id * id;
        const C Z = num * id3;
        const C dZ = (dnum * d + C(3) * num) * id3 * id;  // dZ/deta
        d_RT = k2 * rho * Z;
        d_a = -(k2 * rho * rho);
        d_b = k2 * RT * rho * rho * dZ * C(0.25);
        d_rho = k2 * (RT * (Z + eta * dZ) - C(2) * a_eff * rho) - C(1.0 / 3.0);
    } else {
        // p0 = rho RT/d - a rho^2/q, d = 1 - b rho, q = 1 + 2 b rho - b^2 rho^2
        const C br = b * rho;
        const C d = C(1) - br;
        const C q = C(1) + br * (C(2) - br);
        const C id = recip(d), iq = recip(q);
        d_RT = k2 * rho * id;
        d_a = -(k2 * rho * rho * iq);
        d_b = k2 * rho * rho * (RT * id * id + C(2) * a_eff * rho * d * iq * iq);
        d_rho = k2 * (RT * id * id - C(2) * a_eff * rho * (q - br * d) * iq * iq) - C(1.0 / 3.0);
    }
}

// Transpose of the pull at fluid node (xe, yr): lam_i(x) = dJ/df*_i(x) gathers
// the adjoint of every pulled population that was read from f*_i(x).
//  * x + e_i beyond a wall: node x bounced it back into its own population
//    opposite to i, so lam_i(x) = lb_opp(i)(x).
//  * otherwise node x + e_i pulled it (wrapped with periodic ends, absent past
//    an extrapolated end), and at an extrapolated end the end node of row
//    y + e_iy also read it through the clamped source column.
template <class C>
__device__ inline void gather_lambda(const C* __restrict__ lb, const StepArgs& a, int xe, int yr, C (&lam)[9]) {
    // Branch-free: every population issues two in-range loads (the main source and
    // the clamped-end extra) and selects, so all 18 loads are in flight together.
#define LBM_GATHER(I)                                                                           \
    {                                                                                           \
        int ty = yr + ey(I);                                                                    \
        const bool bounce = !a.yper && (ty < 0 || ty >= a.ny);                                  \
        ty = a.yper ? wrapi(ty, a.ny) : clampi(ty, 0, a.ny - 1);                                \
        int tx = xe + ex(I);                                                                    \
        const bool inx = a.xper || (tx >= 0 && tx < a.nx);                                      \
        tx = a.xper ? wrapi(tx, a.nx) : clampi(tx, 0, a.nx - 1);                                \
        const bool extra = !a.xper && ((ex(I) == 1 && xe == 0) || (ex(I) == -1 && xe == a.nx - 1)); \
        const long long mo = bounce ? (long long)opp(I) * a.plane + (long long)yr * a.pitch + xe \
                                    : (long long)(I) * a.plane + (long long)ty * a.pitch + tx;  \
        const C vm = lb[mo];                                                                    \
        const C ve = lb[(long long)(I) * a.plane + (long long)ty * a.pitch + xe];               \
        lam[I] = bounce ? vm : ((inx ? vm : C(0)) + (extra ? ve : C(0)));                       \
    }
    LBM_GATHER(0) LBM_GATHER(1) LBM_GATHER(2) LBM_GATHER(3) LBM_GATHER(4) LBM_GATHER(5) LBM_GATHER(6)
    LBM_GATHER(7) LBM_GATHER(8)
#undef LBM_GATHER
}

// Interior gather: every x + e_i is a fluid node in range, so lam_i(x) =
// lb_i(x + e_i); gat_off[i] is the uniform byte offset of that source.
template <class C>
__device__ inline void gather_lambda_buf(__amdgpu_buffer_rsrc_t r, const uint32_t (&gat_off)[9], uint32_t node_off,
                                         C (&lam)[9]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) lam[i] = buffer_load<C>(r, node_off, gat_off[i]);
}

// div of a vector field on three rows with the gradient stencil of grad3:
// sum_i 3 w_i e_i . V(x + e_i).
template <class C>
__device__ inline C div3(const Row3<C>& sx, const Row3<C>& mx, const Row3<C>& nx_, const Row3<C>& sy,
                         const Row3<C>& ny_) {
    return C(1.0 / 3.0) * (mx.e - mx.w) + C(1.0 / 12.0) * ((nx_.e - nx_.w) + (sx.e - sx.w)) +
           C(1.0 / 3.0) * (ny_.c - sy.c) + C(1.0 / 12.0) * ((ny_.e + ny_.w) - (sy.e + sy.w));
}

// 4-row tiles with FP32 arithmetic: 8 waves per SIMD (four blocks per compute unit), so
// a 1024 x 256 grid's 1152 blocks take little more than one round.  Without the bound
// the compiler's 102 SGPRs allow seven; with it a few SGPRs move to VGPR lanes
// (measured: the gradient's backward sweep 0.477 -> 0.455 s on that grid).
template <class CD, int TYO>
constexpr int adj_min_waves() { return (sizeof(typename CD::C) == 4 && TYO == 4) ? 8 : 1; }

template <class CD, int EOS, int TYO, int NW>
__global__ __launch_bounds__(64 * NW, (adj_min_waves<CD, TYO>())) void adjoint_kernel(const AdjArgs A) {
    using C = typename CD::C;
    constexpr int H = TYO + 2 * kAdjHalo;
    constexpr int RPT = H / NW;
    static_assert(H % NW == 0, "tile height must be a multiple of the waves per block");
    __shared__ C sRho[H][64], sFx[H][64], sFy[H][64], sPhi[H][64], sLap[H][64];
    __shared__ double sRed[NW][4];

    const StepArgs& a = A.s;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int tile = bid / A.nstrip;
    const int strip = bid - tile * A.nstrip;
    const int y0 = (a.ny >= TYO) ? min(tile * TYO, a.ny - TYO) : 0;
    // the last tile is moved down to end at row ny - 1: its rows below tile * TYO are
    // the previous tile's too, and only that tile adds them to the parameter sums
    const int y_sum = tile * TYO;
    const int x0 = strip * kAdjStripOut;
    const int x = x0 - kAdjHalo + lane;
    const bool xin = x >= 0 && x < a.nx;
    const bool xfl = a.xper || xin;
    int xe = x;
    if (!xin) xe = a.xper ? wrapi(x, a.nx) : clampi(x, 0, a.nx - 1);
    const bool out_lane = lane >= kAdjHalo && lane < 64 - kAdjHalo && xin;
    const int lm = lane > 0 ? lane - 1 : 0, lp = lane < 63 ? lane + 1 : 63;  // edge lanes are halo: clamped, unused

    const C* __restrict__ lb = static_cast<const C*>(A.lam_in);
    C* __restrict__ lout = static_cast<C*>(A.lam_out);
    const C RT = LBM_COEF(C, RT), a_eff = LBM_COEF(C, a_eff), bb = LBM_COEF(C, b);
    const C k2 = LBM_COEF(C, k2), kappa = LBM_COEF(C, kappa);
    const C rho_w = LBM_COEF(C, rho_w), tau = LBM_COEF(C, tau), nu = LBM_COEF(C, nu);
    const C s_e = LBM_COEF(C, s_e), s_eps = LBM_COEF(C, s_eps), s_q = LBM_COEF(C, s_q);
    const C s_j = LBM_COEF(C, s_j), s_v = LBM_COEF(C, s_v);
    const bool walls = !a.yper;

    // Field and adjoint loads through buffer resources (uniform plane offsets in
    // SGPRs).  Interior tiles (every gathered target in range, no wall or end
    // rule) gather lam with uniform offsets too.
    const uint32_t esz = uint32_t(sizeof(C));
    const uint32_t plane_c = uint32_t(a.plane) * esz;
    const __amdgpu_buffer_rsrc_t rfl =
        buffer_rsrc(const_cast<void*>(A.fld), uint32_t(kAdjFieldPlanes) * plane_c + uint32_t(4 * a.nx) * esz);
    const __amdgpu_buffer_rsrc_t rlb = buffer_rsrc(const_cast<C*>(lb), 9u * plane_c);
    const bool tile_inner = (x0 - kAdjHalo - 1 >= 0) && (x0 + 64 - kAdjHalo <= a.nx - 1) &&
                            (y0 - kAdjHalo - 1 >= 0) && (y0 + TYO + kAdjHalo <= a.ny - 1);
    uint32_t gat_off[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) gat_off[i] = uint32_t(i) * plane_c + uint32_t(ey(i) * a.pitch + ex(i)) * esz;

    // ---- phase A: gather lam, the collision's vector-Jacobian product ----------------
    double acc_g = 0.0;
    C fb[RPT][9];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int k = wave + NW * j;
        const int y = y0 - kAdjHalo + k;
        const bool yfl = a.yper || (y >= 0 && y < a.ny);
        const int yr = a.yper ? wrapi(y, a.ny) : y;
#pragma unroll
        for (int i = 0; i < 9; ++i) fb[j][i] = C(0);
        C rho = rho_w, Fbx = C(0), Fby = C(0);
        if (yfl) {
            const uint32_t no = uint32_t(yr * a.pitch + xe) * esz;
            rho = buffer_load<C>(rfl, no, 0);
            if (xfl) {
                const C ux = buffer_load<C>(rfl, no, plane_c), uy = buffer_load<C>(rfl, no, 2 * plane_c);
                const C glx = buffer_load<C>(rfl, no, 3 * plane_c), gly = buffer_load<C>(rfl, no, 4 * plane_c);
                C l[9];
                if (tile_inner)
                    gather_lambda_buf<C>(rlb, gat_off, no, l);
                else
                    gather_lambda<C>(lb, a, xe, yr, l);
                // seeds of J = sum tau_w^2 on the two rows next to each wall: dJ/dtau_w = 2 tau_w, with
                // tau_w = rho_w nu (9 v_x(1/2) - v_x(3/2)) / 3 of this step (written by its forward recompute)
                C vbx = C(0), rbw = C(0), vx = C(0), inv = C(0);
                if (walls && (y <= 1 || y >= a.ny - 2)) {
                    const bool bottom = y <= 1;
                    const int yw = bottom ? 0 : a.ny - 1;  // the row next to the wall
                    const int w = bottom ? y : 3 - (a.ny - 1 - y);
                    const C rw = buffer_load<C>(rfl, uint32_t(yw * a.pitch + xe) * esz, 0);
                    vx = buffer_load<C>(rfl, uint32_t(w * a.nx + xe) * esz, uint32_t(kAdjFieldPlanes) * plane_c);
                    inv = recip(rho);
                    const C tw = C(A.tau_w[(bottom ? 0 : a.nx) + xe]);
                    const C tb = A.seed ? C(A.seed[(bottom ? 0 : a.nx) + xe]) : C(2) * tw;  // dJ/dtau_w
                    if (y == yw) {
                        rbw = tb * tw * recip(rw);  // d tau_w / d rho_w = tau_w / rho_w
                        vbx = tb * rw * nu * C(3);
                    } else {
                        vbx = -(tb * rw * nu * C(1.0 / 3.0));
                    }
                }
                // moments of lam, scaled by the relaxation rates over the squared row norms
                const C A4 = (l[1] + l[2]) + (l[3] + l[4]);
                const C D4 = (l[5] + l[6]) + (l[7] + l[8]);
                const C ne = s_e * C(1.0 / 36.0) * (C(-4) * l[0] - A4 + C(2) * D4);
                const C neps = s_eps * C(1.0 / 36.0) * (C(4) * l[0] - C(2) * A4 + D4);
                const C njx = s_j * C(1.0 / 6.0) * ((l[1] - l[3]) + (l[5] - l[6]) + (l[8] - l[7]));
                const C nqx = s_q * C(1.0 / 12.0) * (C(2) * (l[3] - l[1]) + ((l[5] - l[6]) - (l[7] - l[8])));
                const C njy = s_j * C(1.0 / 6.0) * ((l[2] - l[4]) + (l[5] - l[8]) + (l[6] - l[7]));
                const C nqy = s_q * C(1.0 / 12.0) * (C(2) * (l[4] - l[2]) + ((l[5] + l[6]) - (l[7] + l[8])));
                const C nxx = s_v * C(0.25) * ((l[1] + l[3]) - (l[2] + l[4]));
                const C nxy = s_v * C(0.25) * ((l[5] + l[7]) - (l[6] + l[8]));
                // m_eq = (rho, 3|P|^2/rho - 2 rho, rho - 3|P|^2/rho, Px, -Px, Py, -Py, (Px^2 - Py^2)/rho, Px Py/rho)
                const C u2 = ux * ux + uy * uy;
                C rb = ne * (C(-2) - C(3) * u2) + neps * (C(1) + C(3) * u2) - nxx * (ux * ux - uy * uy) - nxy * (ux * uy);
                const C dee = C(6) * (ne - neps);
                const C Pbx = dee * ux + (njx - nqx) + C(2) * nxx * ux + nxy * uy;
                const C Pby = dee * uy + (njy - nqy) - C(2) * nxx * uy + nxy * ux;
                // P = j + tau F; v = (j + F/2)/rho
                const C jbx = Pbx + vbx * inv, jby = Pby;
                Fbx = tau * Pbx + C(0.5) * vbx * inv;
                Fby = tau * Pby;
                rb += rbw - vbx * vx * inv;
                rb += kappa * (glx * Fbx + gly * Fby);  // F contains kappa rho grad L
                if (k >= kAdjHalo && k < kAdjHalo + TYO && out_lane && y < a.ny) {
                    if (y >= y_sum) acc_g += double(Fbx);
                    // f~ = lam - M^T (D M lam) + rho~ + e . j~ (rho~ gets the stencil terms in phase E)
                    const C c0 = -ne - C(2) * neps, c1 = C(2) * ne + neps;
                    const C X = njx - C(2) * nqx, Y = njy - C(2) * nqy, Xd = njx + nqx, Yd = njy + nqy;
                    fb[j][0] = l[0] - C(4) * (neps - ne) + rb;
                    fb[j][1] = l[1] - (c0 + X + nxx) + rb + jbx;
                    fb[j][3] = l[3] - (c0 - X + nxx) + rb - jbx;
                    fb[j][2] = l[2] - (c0 + Y - nxx) + rb + jby;
                    fb[j][4] = l[4] - (c0 - Y - nxx) + rb - jby;
                    fb[j][5] = l[5] - (c1 + Xd + Yd + nxy) + rb + jbx + jby;
                    fb[j][7] = l[7] - (c1 - Xd - Yd + nxy) + rb - jbx - jby;
                    fb[j][6] = l[6] - (c1 - Xd + Yd - nxy) + rb - jbx + jby;
                    fb[j][8] = l[8] - (c1 + Xd - Yd - nxy) + rb + jbx - jby;
                }
            }
        }
        sRho[k][lane] = rho;  // ghost rows hold rho_w, ghost columns the copied end column
        sFx[k][lane] = Fbx;   // zero off the fluid
        sFy[k][lane] = Fby;
    }
    __syncthreads();

    // ---- phase D: phi~ = div F~, L~ = -div(kappa rho F~) on rows 1 .. H-2 -----------
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int k = wave + NW * j;
        if (k < 1 || k > H - 2) continue;
        const Row3<C> sx{sFx[k - 1][lane], sFx[k - 1][lp], sFx[k - 1][lm]};
        const Row3<C> mx{sFx[k][lane], sFx[k][lp], sFx[k][lm]};
        const Row3<C> nx_{sFx[k + 1][lane], sFx[k + 1][lp], sFx[k + 1][lm]};
        const Row3<C> sy{sFy[k - 1][lane], sFy[k - 1][lp], sFy[k - 1][lm]};
        const Row3<C> ny_{sFy[k + 1][lane], sFy[k + 1][lp], sFy[k + 1][lm]};
        sPhi[k][lane] = div3(sx, mx, nx_, sy, ny_);
#define LBM_G(F, kk, ll) (kappa * sRho[kk][ll] * F[kk][ll])
        const Row3<C> gsx{LBM_G(sFx, k - 1, lane), LBM_G(sFx, k - 1, lp), LBM_G(sFx, k - 1, lm)};
        const Row3<C> gmx{LBM_G(sFx, k, lane), LBM_G(sFx, k, lp), LBM_G(sFx, k, lm)};
        const Row3<C> gnx{LBM_G(sFx, k + 1, lane), LBM_G(sFx, k + 1, lp), LBM_G(sFx, k + 1, lm)};
        const Row3<C> gsy{LBM_G(sFy, k - 1, lane), LBM_G(sFy, k - 1, lp), LBM_G(sFy, k - 1, lm)};
        const Row3<C> gny{LBM_G(sFy, k + 1, lane), LBM_G(sFy, k + 1, lp), LBM_G(sFy, k + 1, lm)};
#undef LBM_G
        sLap[k][lane] = -div3(gsx, gmx, gnx, gsy, gny);
    }
    __syncthreads();

    // ---- phase E: rho~, dJ/df of the outputs, parameter sums ------------------------
    double acc_rt = 0.0, acc_a = 0.0, acc_b = 0.0;
    auto rho_bar_at = [&](int k, int l2, C& dRT, C& dA, C& dB) {
        // lap(L~) + phi'(rho) phi~ at tile position (k, l2); returns the EOS partials too.  Past
        // the tile's edge lanes (only reached from a ghost column two nodes beyond an
        // extrapolated end) L~ is zero, as it is in the clamped edge lane.
        const int l2m = l2 > 0 ? l2 - 1 : 0, l2p = l2 < 63 ? l2 + 1 : 63;
        const Row3<C> s{sLap[k - 1][l2], sLap[k - 1][l2p], sLap[k - 1][l2m]};
        const Row3<C> m{sLap[k][l2], sLap[k][l2p], sLap[k][l2m]};
        const Row3<C> n{sLap[k + 1][l2], sLap[k + 1][l2p], sLap[k + 1][l2m]};
        C dr;
        phi_partials<EOS, C>(sRho[k][l2], RT, a_eff, bb, k2, dr, dRT, dA, dB);
        return lap3(s, m, n) + dr * sPhi[k][l2];
    };
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int k = wave + NW * j;
        const int y = y0 - kAdjHalo + k;
        if (k < kAdjHalo || k >= kAdjHalo + TYO || !out_lane || y >= a.ny) continue;  // y < ny: fluid row
        C dRT, dA, dB;
        C rb = rho_bar_at(k, lane, dRT, dA, dB);
        const C ph = sPhi[k][lane];
        const bool sums = y >= y_sum;
        if (sums) {
            acc_rt += double(ph * dRT);
            acc_a += double(ph * dA);
            acc_b += double(ph * dB);
        }
        if (!a.xper && (x == 0 || x == a.nx - 1)) {
            // ghost columns copy this end column: their adjoints add back here
            const int sgn = x == 0 ? -1 : 1;
            C t0, t1, t2;
            rb += rho_bar_at(k, lane + sgn, t0, t1, t2);
            rb += rho_bar_at(k, lane + 2 * sgn, t0, t1, t2);
        }
        const bool edge = sums && ((!a.yper && (y == 0 || y == a.ny - 1)) || (!a.xper && (x == 0 || x == a.nx - 1)));
        if (edge) {
            // ghost positions next to the domain whose nearest node is this one: their phi
            // depends on the parameters (wall rows at the fixed rho_w, end columns at copies)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int zx = x + dx, zy = y + dy;
                    const bool zyf = a.yper || (zy >= 0 && zy < a.ny);
                    const bool zxf = a.xper || (zx >= 0 && zx < a.nx);
                    if (zyf && zxf) continue;
                    const int px = a.xper ? wrapi(zx, a.nx) : clampi(zx, 0, a.nx - 1);
                    const int py = a.yper ? wrapi(zy, a.ny) : clampi(zy, 0, a.ny - 1);
                    if (px != x || py != y) continue;
                    C dr, tRT, tA, tB;
                    phi_partials<EOS, C>(sRho[k + dy][lane + dx], RT, a_eff, bb, k2, dr, tRT, tA, tB);
                    const C pz = sPhi[k + dy][lane + dx];
                    acc_rt += double(pz * tRT);
                    acc_a += double(pz * tA);
                    acc_b += double(pz * tB);
                }
        }
        const long long o = (long long)y * a.pitch + x;
#pragma unroll
        for (int i = 0; i < 9; ++i) lout[(long long)i * a.plane + o] = fb[j][i] + rb;
    }

    // ---- block sums of the parameter adjoints (fixed order) ----------------------
    const double r0 = wave_sum(acc_g), r1 = wave_sum(acc_rt), r2 = wave_sum(acc_a), r3 = wave_sum(acc_b);
    if (lane == 0) {
        sRed[wave][0] = r0;
        sRed[wave][1] = r1;
        sRed[wave][2] = r2;
        sRed[wave][3] = r3;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += sRed[w][threadIdx.x];
        A.partial[(long long)blockIdx.x * 4 + threadIdx.x] = t;
    }
}

// Parameter sums of a run of adjoint launches (consecutive steps, in the order
// they ran): stage 1 sums each launch's block partials in a fixed order (one
// block per launch), stage 2 adds the launch totals to acc[0..3] one after
// another.  acc therefore receives the same additions in the same order
// whatever the grouping of launches into runs, so the result does not depend
// on the checkpoint segment length.
constexpr int kAdjRedThreads = 256;
__global__ __launch_bounds__(kAdjRedThreads) void adjoint_reduce_stage1(const double* __restrict__ partial, int blocks,
                                                                        double* __restrict__ red) {
    __shared__ double sh[4][kAdjRedThreads];
    const int t = threadIdx.x;
    const double* p = partial + (long long)blockIdx.x * blocks * 4;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = t; i < blocks; i += kAdjRedThreads)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += p[i * 4 + q];
#pragma unroll
    for (int q = 0; q < 4; ++q) sh[q][t] = v[q];
    __syncthreads();
    for (int s = kAdjRedThreads / 2; s > 0; s >>= 1) {
        if (t < s)
#pragma unroll
            for (int q = 0; q < 4; ++q) sh[q][t] += sh[q][t + s];
        __syncthreads();
    }
    if (t < 4) red[blockIdx.x * 4 + t] = sh[t][0];
}

__global__ void adjoint_reduce_stage2(const double* __restrict__ red, int launches, double* __restrict__ acc) {
    const int q = threadIdx.x;
    if (q >= 4) return;
    double a = acc[q];
    for (int r = 0; r < launches; ++r) a += red[r * 4 + q];
    acc[q] = a;
}

// dJ/df* of the initial state: the pull transpose of the last adjoint step's
// output, as FP64 [9][ny][nx].
template <class C>
__global__ void adjoint_gather_kernel(const C* __restrict__ lb, const StepArgs a, double* __restrict__ out) {
    const long long n = (long long)a.nx * a.ny;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        const int y = int(c / a.nx), x = int(c - (long long)y * a.nx);
        C lam[9];
        gather_lambda<C>(lb, a, x, y, lam);
#pragma unroll
        for (int i = 0; i < 9; ++i) out[(long long)i * n + c] = double(lam[i]);
    }
}

template <class CD, int EOS, int TYO, int NW>
hipError_t launch_adj_t(const AdjArgs& A, hipStream_t s) {
    const dim3 grid(A.nstrip * ((A.s.ny + TYO - 1) / TYO)), block(64 * NW);
    hipLaunchKernelGGL((adjoint_kernel<CD, EOS, TYO, NW>), grid, block, 0, s, A);
    return hipGetLastError();
}

template <class CD, int EOS>
hipError_t launch_adj_e(const AdjArgs& A, hipStream_t s) {
    if (A.waves != 8) return hipErrorInvalidValue;
    switch (A.ty) {
        case 4: return launch_adj_t<CD, EOS, 4, 8>(A, s);
        case 12: return launch_adj_t<CD, EOS, 12, 8>(A, s);
        default: return hipErrorInvalidValue;
    }
}

// The forward step of the backward sweep's recompute: the tile step (8-row,
// 4-wave tiles) that also writes the adjoint's fields of the step.
template <class CD, int EOS>
__global__ __launch_bounds__(256) void tile_save_kernel(const StepArgs a) {
    tile_body<CD, EOS, false, 8, 4, true>(a, a.fin, a.fout, a.tau_w, a.p_w, a.dtau_w, xcd_remap(blockIdx.x, gridDim.x),
                                          0);
}

template <class CD>
hipError_t launch_save_c(const StepArgs& a, int eos, hipStream_t s) {
    StepArgs b = a;
    b.nstrip = (a.nx + kStripOut - 1) / kStripOut;
    const dim3 grid(b.nstrip * ((a.ny + 7) / 8)), block(256);
    if (eos == LBM_EOS_CS)
        hipLaunchKernelGGL((tile_save_kernel<CD, LBM_EOS_CS>), grid, block, 0, s, b);
    else
        hipLaunchKernelGGL((tile_save_kernel<CD, LBM_EOS_PR>), grid, block, 0, s, b);
    return hipGetLastError();
}

template <class CD>
hipError_t launch_adj_c(const AdjArgs& A, int eos, hipStream_t s) {
    return eos == LBM_EOS_CS ? launch_adj_e<CD, LBM_EOS_CS>(A, s) : launch_adj_e<CD, LBM_EOS_PR>(A, s);
}

}  // namespace

hipError_t launch_adjoint(const AdjArgs& A, int storage, int eos, hipStream_t s) {
    switch (storage) {
        case LBM_F64: return launch_adj_c<CodecF64>(A, eos, s);
        case LBM_F32: return launch_adj_c<CodecF32>(A, eos, s);
        case LBM_F32D: return launch_adj_c<CodecF32D>(A, eos, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_save(const StepArgs& a, int storage, int eos, hipStream_t s) {
    if (!a.save) return hipErrorInvalidValue;
    switch (storage) {
        case LBM_F64: return launch_save_c<CodecF64>(a, eos, s);
        case LBM_F32: return launch_save_c<CodecF32>(a, eos, s);
        case LBM_F32D: return launch_save_c<CodecF32D>(a, eos, s);
        default: return hipErrorInvalidValue;
    }
}

namespace {
// One block per step: the largest tau_w^2 over both walls (lane-strided, then wave
// butterflies, then the waves in order; ties go to the smaller index w nx + x).
constexpr int kSeedThreads = 256;
__global__ __launch_bounds__(kSeedThreads) void peak_seed_kernel(const double* __restrict__ tau_w,
                                                                 double* __restrict__ seed, int nx) {
    __shared__ double sv[kSeedThreads / 64], si[kSeedThreads / 64];
    const long long base = (long long)blockIdx.x * 2 * nx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v = -1.0, idx = 1e300;
    for (int i = threadIdx.x; i < 2 * nx; i += kSeedThreads) {
        const double t = tau_w[base + i];
        const double t2 = t * t;
        if (t2 > v || (t2 == v && double(i) < idx)) { v = t2; idx = double(i); }
        seed[base + i] = 0.0;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64), oi = __shfl_xor(idx, off, 64);
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    if (lane == 0) { sv[wave] = v; si[wave] = idx; }
    __syncthreads();  // also orders the zero fill before the seed store below
    if (threadIdx.x != 0) return;
    for (int w = 1; w < kSeedThreads / 64; ++w)
        if (sv[w] > v || (sv[w] == v && si[w] < idx)) { v = sv[w]; idx = si[w]; }
    if (!(v >= 0.0)) return;  // every tau_w NaN: no seed
    const int i = int(idx);
    seed[base + i] = 2.0 * tau_w[base + i];
}
}  // namespace

hipError_t launch_peak_seed(const double* tau_w, double* seed, int nx, int steps, hipStream_t s) {
    if (steps <= 0) return hipSuccess;
    hipLaunchKernelGGL(peak_seed_kernel, dim3(steps), dim3(kSeedThreads), 0, s, tau_w, seed, nx);
    return hipGetLastError();
}

hipError_t launch_adjoint_reduce(const double* partial, int launches, int blocks, double* red, double* acc,
                                 hipStream_t s) {
    if (launches <= 0) return hipSuccess;
    hipLaunchKernelGGL(adjoint_reduce_stage1, dim3(launches), dim3(kAdjRedThreads), 0, s, partial, blocks, red);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(adjoint_reduce_stage2, dim3(1), dim3(64), 0, s, red, launches, acc);
    return hipGetLastError();
}

hipError_t launch_adjoint_gather(const void* lam, const StepArgs& a, int storage, double* out, hipStream_t s) {
    const long long n = (long long)a.nx * a.ny;
    const int blocks = int((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048);
    switch (storage) {
        case LBM_F64:
        case LBM_F32D:
            hipLaunchKernelGGL(adjoint_gather_kernel<double>, dim3(blocks), dim3(256), 0, s,
                               static_cast<const double*>(lam), a, out);
            break;
        case LBM_F32:
            hipLaunchKernelGGL(adjoint_gather_kernel<float>, dim3(blocks), dim3(256), 0, s,
                               static_cast<const float*>(lam), a, out);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int adjoint_blocks(int nx, int ny, int ty) {
    return ((nx + kAdjStripOut - 1) / kAdjStripOut) * ((ny + ty - 1) / ty);
}

}  // namespace lbm
