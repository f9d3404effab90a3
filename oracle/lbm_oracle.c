/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY (see lbm_oracle.h).
 *
 * A plain FP64 CPU time stepper for the EOS-based multiphase MRT lattice
 * Boltzmann method of arXiv 2103.08301, Sec. 2.  Each stage of the step is a
 * separate loop over the whole grid writing a whole-grid array, in the order
 * stream -> moments -> EOS field -> Laplacian -> force -> velocities ->
 * collision -> wall diagnostics, so that every stage can be read against the
 * paper on its own.  There is no blocking, fusion or reordering.
 *
 * Where the paper is silent or garbled the following readings are taken
 * (each is also listed with its justification in the design notes):
 *  - D2Q9 velocities/weights are the standard ones; the symbols are lost in
 *    the text after eq. 2.1 but the coefficients 3, 9/2, 3/2 of eq. 2.2 fix
 *    c_s^2 = 1/3.
 *  - The relaxation rates after eq. 2.1 are positive (eq. 2.1 already carries
 *    the minus sign); M is the Lallemand-Luo moment basis in the order
 *    (rho, e, eps, jx, qx, jy, qy, pxx, pxy) implied by the pattern of S.
 *  - The momentum rows relax at s_j = 1/tau so that the velocity shift of
 *    Sec. 2.2 (u_eq = u + tau F / rho) adds exactly F to the momentum.
 *  - Gradients and Laplacians are the isotropic D2Q9-weighted differences
 *    grad = 3 sum w_i e_i psi(x+e_i), lap = 6 sum w_i (psi(x+e_i) - psi(x)).
 *  - The k scaling of eqs. 2.13-2.17 is applied in mesh units:
 *    F = -grad(k^2 p0 - rho/3) + kappa rho grad(lap rho).
 *  - PR alpha(T) uses the standard kappa_w = 0.37464 + 1.54226 w - 0.26992 w^2.
 *  - Walls: halfway bounce-back at y = -1/2 and y = ny - 1/2; ghost rows carry
 *    a virtual wall density rho_w (wettability).  Ends: extrapolated
 *    (zero-gradient copy of the boundary column) or periodic.
 *  - Pressure drop: uniform body force density dp/nx along +x.
 *  - Wall shear: tau_w = rho nu dv_x/ds from the quadratic through v(0)=0,
 *    v(1/2), v(3/2); wall pressure: isotropic part of eq. 2.8 at the first row.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* D2Q9 lattice (standard; see the reading above).                          */

static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* Lallemand-Luo moment matrix; rows rho, e, eps, jx, qx, jy, qy, pxx, pxy. */
static const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

/* M^-1 = M^T diag(1/|row_k|^2): the rows of M are mutually orthogonal. */
static void inverse_moment_matrix(double Minv[9][9]) {
    for (int k = 0; k < 9; ++k) {
        double n2 = 0.0;
        for (int j = 0; j < 9; ++j) n2 += MM[k][j] * MM[k][j];
        for (int i = 0; i < 9; ++i) Minv[i][k] = MM[k][i] / n2;
    }
}

void orc_velocities(int i, int* ex, int* ey, double* w) {
    *ex = EX[i];
    *ey = EY[i];
    *w = WT[i];
}

void orc_moment_matrix(double* M81) {
    for (int k = 0; k < 9; ++k)
        for (int i = 0; i < 9; ++i) M81[k * 9 + i] = MM[k][i];
}

/* Eq. 2.2. */
void orc_equilibrium(double rho, double ux, double uy, double* feq) {
    double usq = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double eu = EX[i] * ux + EY[i] * uy;
        feq[i] = rho * WT[i] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
    }
}

/* ------------------------------------------------------------------------ */
/* Equation of state.  Both EOS are written p0 = R T G(rho) - a A(T) H(rho)   */
/* with A = 1 (CS) or alpha(T) (PR), so the critical point follows from G, H.*/

typedef struct {
    int kind;
    double a, b, R, T, A;
} eos_t;

/* G and H with first and second derivatives in rho. */
static void eos_GH(int kind, double b, double rho, double G[3], double H[3]) {
    if (kind == ORC_EOS_CS) {
        /* Carnahan-Starling repulsion with van der Waals attraction:
           p0 = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2, eta = b rho / 4. */
        double c = b / 4.0, eta = c * rho, D = 1.0 - eta;
        double N = 1.0 + eta + eta * eta - eta * eta * eta;
        double N1 = 1.0 + 2.0 * eta - 3.0 * eta * eta;
        double N2 = 2.0 - 6.0 * eta;
        double D3 = D * D * D, D4 = D3 * D, D5 = D4 * D;
        double Z = N / D3;
        double Z1 = N1 / D3 + 3.0 * N / D4;
        double Z2 = N2 / D3 + 6.0 * N1 / D4 + 12.0 * N / D5;
        G[0] = rho * Z;
        G[1] = Z + eta * Z1;
        G[2] = c * (2.0 * Z1 + eta * Z2);
        H[0] = rho * rho;
        H[1] = 2.0 * rho;
        H[2] = 2.0;
    } else {
        /* Peng-Robinson, eq. 2.18. */
        double D = 1.0 - b * rho;
        double Q = 1.0 + 2.0 * b * rho - b * b * rho * rho;
        double Q1 = 2.0 * b - 2.0 * b * b * rho;
        double Q2 = -2.0 * b * b;
        G[0] = rho / D;
        G[1] = 1.0 / (D * D);
        G[2] = 2.0 * b / (D * D * D);
        H[0] = rho * rho / Q;
        H[1] = 2.0 * rho / Q - rho * rho * Q1 / (Q * Q);
        H[2] = 2.0 / Q - 4.0 * rho * Q1 / (Q * Q) - rho * rho * Q2 / (Q * Q)
             + 2.0 * rho * rho * Q1 * Q1 / (Q * Q * Q);
    }
}

static double eos_rho_max(int kind, double b) {
    return kind == ORC_EOS_CS ? 4.0 / b : 1.0 / b;
}

static double eos_p(const eos_t* e, double rho, int order) {
    double G[3], H[3];
    eos_GH(e->kind, e->b, rho, G, H);
    return e->R * e->T * G[order] - e->a * e->A * H[order];
}

/* Critical point: dp/drho = d2p/drho2 = 0.  Because p0 is linear in R T at
   fixed A(Tc) = 1, eliminating T leaves G'H'' - G''H' = 0 in rho alone. */
static int eos_critical(int kind, double a, double b, double R, double* rho_c, double* T_c) {
    if (!(a > 0 && b > 0 && R > 0)) return ORC_EINVAL;
    double rmax = eos_rho_max(kind, b);
    const int N = 20000;
    double prev_r = 0.0, prev_c = 0.0;
    int found = 0;
    double lo = 0, hi = 0;
    for (int k = 1; k < N; ++k) {
        double r = rmax * k / N;
        double G[3], H[3];
        eos_GH(kind, b, r, G, H);
        double c = G[1] * H[2] - G[2] * H[1];
        if (k > 1 && prev_c > 0 && c <= 0) {
            lo = prev_r;
            hi = r;
            found = 1;
            break;
        }
        prev_r = r;
        prev_c = c;
    }
    if (!found) return ORC_EINVAL;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double G[3], H[3];
        eos_GH(kind, b, mid, G, H);
        double c = G[1] * H[2] - G[2] * H[1];
        if (c > 0) lo = mid; else hi = mid;
    }
    double rc = 0.5 * (lo + hi);
    double G[3], H[3];
    eos_GH(kind, b, rc, G, H);
    *rho_c = rc;
    *T_c = a * H[1] / (R * G[1]);
    return ORC_OK;
}

double orc_alpha(const orc_params* p, double T, double T_c) {
    if (p->eos != ORC_EOS_PR) return 1.0;
    double kw = 0.37464 + 1.54226 * p->omega - 0.26992 * p->omega * p->omega;
    double s = 1.0 + kw * (1.0 - sqrt(T / T_c));
    return s * s;
}

static int eos_at(const orc_params* p, double T, eos_t* e) {
    double rc, Tc;
    int st = eos_critical(p->eos, p->a, p->b, p->R, &rc, &Tc);
    if (st) return st;
    e->kind = p->eos;
    e->a = p->a;
    e->b = p->b;
    e->R = p->R;
    e->T = T;
    e->A = orc_alpha(p, T, Tc);
    return ORC_OK;
}

int orc_critical(const orc_params* p, double* rho_c, double* T_c) {
    return eos_critical(p->eos, p->a, p->b, p->R, rho_c, T_c);
}

double orc_p0(const orc_params* p, double T, double rho) {
    eos_t e;
    if (eos_at(p, T, &e)) return NAN;
    return eos_p(&e, rho, 0);
}

double orc_dp0(const orc_params* p, double T, double rho, int order) {
    eos_t e;
    if (order < 1 || order > 2 || eos_at(p, T, &e)) return NAN;
    return eos_p(&e, rho, order);
}

/* Root of p0(rho) = target on [lo, hi], where p0 is monotone increasing. */
static double eos_solve(const eos_t* e, double target, double lo, double hi) {
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (eos_p(e, mid, 0) < target) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Equal-area integral of Sec. 2.2 (Maxwell construction) in the density
   variable: integral_{rho_g}^{rho_l} (p0 - p*) / rho^2 d rho, evaluated with the
   substitution s = ln rho and composite 5-point Gauss-Legendre quadrature. */
static double maxwell_area(const eos_t* e, double pstar, double rg, double rl) {
    static const double gx[5] = {-0.9061798459386640, -0.5384693101056831, 0.0,
                                 0.5384693101056831, 0.9061798459386640};
    static const double gw[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                                 0.4786286704993665, 0.2369268850561891};
    const int panels = 400;
    double s0 = log(rg), s1 = log(rl), hs = (s1 - s0) / panels, sum = 0.0;
    for (int k = 0; k < panels; ++k) {
        double c = s0 + (k + 0.5) * hs;
        for (int q = 0; q < 5; ++q) {
            double rho = exp(c + 0.5 * hs * gx[q]);
            sum += gw[q] * (eos_p(e, rho, 0) - pstar) / rho;
        }
    }
    return sum * 0.5 * hs;
}

int orc_coexistence(const orc_params* p, double T, double* rho_g, double* rho_l, double* p_star) {
    eos_t e;
    int st = eos_at(p, T, &e);
    if (st) return st;
    double rmax = eos_rho_max(p->eos, p->b);
    /* Spinodals: the local maximum (gas side) and local minimum (liquid side) of p0. */
    const int N = 200000;
    double sg = -1, sl = -1, prev = eos_p(&e, rmax / N, 1);
    for (int k = 2; k < N; ++k) {
        double r = rmax * k / N, d = eos_p(&e, r, 1);
        if (sg < 0 && prev > 0 && d <= 0) sg = r;
        if (sg > 0 && prev < 0 && d >= 0) { sl = r; break; }
        prev = d;
    }
    if (sg < 0 || sl < 0) return ORC_EINVAL; /* at or above the critical temperature */
    /* refine both spinodals by bisection on dp/drho */
    double lo = sg - rmax / N, hi = sg;
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (lo + hi);
        if (m <= lo || m >= hi) break;
        if (eos_p(&e, m, 1) > 0) lo = m; else hi = m;
    }
    sg = lo;
    lo = sl - rmax / N;
    hi = sl;
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (lo + hi);
        if (m <= lo || m >= hi) break;
        if (eos_p(&e, m, 1) < 0) lo = m; else hi = m;
    }
    sl = hi;
    double p_hi = eos_p(&e, sg, 0);
    double p_lo = eos_p(&e, sl, 0);
    if (p_lo <= 0) p_lo = p_hi * 1e-300;
    double rg = 0, rl = 0, pm = 0;
    for (int it = 0; it < 2000; ++it) {
        pm = (p_hi > 4.0 * p_lo) ? sqrt(p_lo * p_hi) : 0.5 * (p_lo + p_hi);
        if (pm <= p_lo || pm >= p_hi) break;
        rg = eos_solve(&e, pm, 0.0, sg);
        rl = eos_solve(&e, pm, sl, rmax);
        double A = maxwell_area(&e, pm, rg, rl);
        if (A > 0) p_lo = pm; else p_hi = pm;
    }
    pm = 0.5 * (p_lo + p_hi);
    *rho_g = eos_solve(&e, pm, 0.0, sg);
    *rho_l = eos_solve(&e, pm, sl, rmax);
    *p_star = pm;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Stencils on an arbitrary row-major array with row pitch `pitch`.          */

/* grad psi = (1/c_s^2) sum_i w_i e_i psi(x + e_i), c_s^2 = 1/3 */
static void grad_at(const double* c, long pitch, double* gx, double* gy) {
    double sx = 0.0, sy = 0.0;
    for (int i = 1; i < 9; ++i) {
        double v = c[EY[i] * pitch + EX[i]];
        sx += WT[i] * EX[i] * v;
        sy += WT[i] * EY[i] * v;
    }
    *gx = 3.0 * sx;
    *gy = 3.0 * sy;
}

/* lap psi = (2/c_s^2) sum_i w_i (psi(x + e_i) - psi(x)) */
static double lap_at(const double* c, long pitch) {
    double s = 0.0;
    for (int i = 1; i < 9; ++i) s += WT[i] * (c[EY[i] * pitch + EX[i]] - c[0]);
    return 6.0 * s;
}

void orc_grad_field(const double* a, int w, int h, double* gx, double* gy) {
    for (int y = 1; y < h - 1; ++y)
        for (int x = 1; x < w - 1; ++x)
            grad_at(a + (long)y * w + x, w, gx + (long)(y - 1) * (w - 2) + (x - 1),
                    gy + (long)(y - 1) * (w - 2) + (x - 1));
}

void orc_lap_field(const double* a, int w, int h, double* lap) {
    for (int y = 1; y < h - 1; ++y)
        for (int x = 1; x < w - 1; ++x)
            lap[(long)(y - 1) * (w - 2) + (x - 1)] = lap_at(a + (long)y * w + x, w);
}

/* ------------------------------------------------------------------------ */
/* MRT collision with the velocity-shift forcing of Sec. 2.2.               */

typedef struct {
    double S[9];     /* diagonal relaxation rates */
    double tau;
    int forcing;     /* ORC_FORCING_* */
    double Minv[9][9];
} collide_t;

static void collide_setup(const orc_params* p, collide_t* c) {
    double sv = 1.0 / p->tau;
    double sj = p->s_j > 0 ? p->s_j : sv;
    double S[9] = {0.0, p->s_e, p->s_eps, sj, p->s_q, sj, p->s_q, sv, sv};
    memcpy(c->S, S, sizeof S);
    c->tau = p->tau;
    c->forcing = p->forcing;
    inverse_moment_matrix(c->Minv);
}

/* f -> f* for one node given the force; also returns rho and v = u + F/(2 rho).
   Velocity shift (the method): the equilibrium is taken at u + tau F/rho.
   Exact difference (comparison only): the equilibrium is taken at u and the
   difference f_eq(rho, u + F/rho) - f_eq(rho, u) is added after the collision. */
static void collide(const collide_t* c, const double* f, double Fx, double Fy,
                    double* fout, double* rho_out, double* vx, double* vy) {
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) {
        rho += f[i];
        jx += f[i] * EX[i];
        jy += f[i] * EY[i];
    }
    double ux = jx / rho, uy = jy / rho;
    const int edm = c->forcing == ORC_FORCING_EXACT_DIFFERENCE;
    double uex = edm ? ux : ux + c->tau * Fx / rho, uey = edm ? uy : uy + c->tau * Fy / rho;
    *vx = ux + Fx / (2.0 * rho);
    *vy = uy + Fy / (2.0 * rho);
    *rho_out = rho;
    double feq[9], m[9], meq[9], ms[9];
    orc_equilibrium(rho, uex, uey, feq);
    for (int k = 0; k < 9; ++k) {
        m[k] = 0.0;
        meq[k] = 0.0;
        for (int i = 0; i < 9; ++i) {
            m[k] += MM[k][i] * f[i];
            meq[k] += MM[k][i] * feq[i];
        }
        ms[k] = m[k] - c->S[k] * (m[k] - meq[k]);
    }
    for (int i = 0; i < 9; ++i) {
        fout[i] = 0.0;
        for (int k = 0; k < 9; ++k) fout[i] += c->Minv[i][k] * ms[k];
    }
    if (edm) {
        double f1[9];
        orc_equilibrium(rho, ux + Fx / rho, uy + Fy / rho, f1);
        for (int i = 0; i < 9; ++i) fout[i] += f1[i] - feq[i];
    }
}

void orc_collide_node(const orc_params* p, const double* f9, double Fx, double Fy,
                      double* fout9, double* rho, double* vx, double* vy) {
    collide_t c;
    collide_setup(p, &c);
    collide(&c, f9, Fx, Fy, fout9, rho, vx, vy);
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the state advances by the   */
/* odd constant 0x9E3779B97F4A7C15 and each output is a mix of the state.    */

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

uint64_t orc_splitmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------ */
/* Time stepper.                                                            */

struct orc_sim {
    int nx, ny;
    orc_params p;
    eos_t eos;
    collide_t col;
    double T, Tc, rho_g, rho_l, rho_w;
    double *f, *fs;                 /* [9][ny][nx] post-collision state, streamed */
    double *rho, *jx, *jy;          /* [ny][nx] */
    double *rext, *phiext;          /* [ny+4][nx+4], ghost ring of width 2 */
    double *lap;                    /* [ny+2][nx+2], ring of width 1 */
    double *Fx, *Fy, *vx, *vy;      /* [ny][nx] */
    double *tau_w, *p_w;            /* [2][nx] */
    orc_summary* hist;
    int64_t hist_n, hist_cap;
    int64_t step, unstable_step;
    double int_peak_tau2, int_tau2;
    double run[4][2];               /* running extremes: tau max, tau min, p max, p min per wall */
};

void orc_params_default(orc_params* p) {
    memset(p, 0, sizeof *p);
    p->eos = ORC_EOS_CS;
    p->a = 1.0;
    p->b = 4.0;
    p->R = 1.0;
    p->omega = 0.344;
    p->T_over_Tc = 0.85;
    p->k = 1.0;
    p->kappa = 0.001;
    p->tau = 1.0;
    p->s_e = 1.64;
    p->s_eps = 1.54;
    p->s_q = 1.7;
    p->s_j = 0.0;
    p->rho_wall = NAN;
    p->dp = 0.0;
    p->x_periodic = 0;
    p->y_periodic = 0;
    p->check_every = 1000;
    p->v_limit = 0.5;
    p->forcing = ORC_FORCING_VELOCITY_SHIFT;
}

int orc_create(int nx, int ny, const orc_params* p, orc_sim** out) {
    *out = NULL;
    if (nx < 3 || ny < 3 || !(p->tau > 0.5) || p->check_every < 1 ||
        (p->forcing != ORC_FORCING_VELOCITY_SHIFT && p->forcing != ORC_FORCING_EXACT_DIFFERENCE))
        return ORC_EINVAL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof *s);
    if (!s) return ORC_ENOMEM;
    s->nx = nx;
    s->ny = ny;
    s->p = *p;
    double rc;
    int st = eos_critical(p->eos, p->a, p->b, p->R, &rc, &s->Tc);
    if (st) { free(s); return st; }
    s->T = p->T_over_Tc * s->Tc;
    st = eos_at(p, s->T, &s->eos);
    if (st) { free(s); return st; }
    if (p->T_over_Tc < 1.0) {
        double ps;
        st = orc_coexistence(p, s->T, &s->rho_g, &s->rho_l, &ps);
        if (st) { free(s); return st; }
    } else {
        s->rho_g = s->rho_l = NAN;
    }
    s->rho_w = isnan(p->rho_wall) ? s->rho_l : p->rho_wall;
    collide_setup(p, &s->col);
    long n = (long)nx * ny;
    s->f = (double*)calloc(9 * n, sizeof(double));
    s->fs = (double*)calloc(9 * n, sizeof(double));
    s->rho = (double*)calloc(n, sizeof(double));
    s->jx = (double*)calloc(n, sizeof(double));
    s->jy = (double*)calloc(n, sizeof(double));
    s->rext = (double*)calloc((long)(nx + 4) * (ny + 4), sizeof(double));
    s->phiext = (double*)calloc((long)(nx + 4) * (ny + 4), sizeof(double));
    s->lap = (double*)calloc((long)(nx + 2) * (ny + 2), sizeof(double));
    s->Fx = (double*)calloc(n, sizeof(double));
    s->Fy = (double*)calloc(n, sizeof(double));
    s->vx = (double*)calloc(n, sizeof(double));
    s->vy = (double*)calloc(n, sizeof(double));
    s->tau_w = (double*)calloc(2 * (long)nx, sizeof(double));
    s->p_w = (double*)calloc(2 * (long)nx, sizeof(double));
    if (!s->f || !s->fs || !s->rho || !s->jx || !s->jy || !s->rext || !s->phiext || !s->lap ||
        !s->Fx || !s->Fy || !s->vx || !s->vy || !s->tau_w || !s->p_w) {
        orc_destroy(s);
        return ORC_ENOMEM;
    }
    s->unstable_step = -1;
    *out = s;
    return ORC_OK;
}

void orc_destroy(orc_sim* s) {
    if (!s) return;
    free(s->f); free(s->fs); free(s->rho); free(s->jx); free(s->jy);
    free(s->rext); free(s->phiext); free(s->lap);
    free(s->Fx); free(s->Fy); free(s->vx); free(s->vy);
    free(s->tau_w); free(s->p_w); free(s->hist);
    free(s);
}

int orc_state(const orc_sim* s, double* T, double* Tc, double* rho_g, double* rho_l, double* rho_w) {
    *T = s->T;
    *Tc = s->Tc;
    *rho_g = s->rho_g;
    *rho_l = s->rho_l;
    *rho_w = s->rho_w;
    return ORC_OK;
}

#define FI(s, arr, i, y, x) ((arr)[((long)(i) * (s)->ny + (y)) * (s)->nx + (x)])
#define CI(s, y, x) ((long)(y) * (s)->nx + (x))
#define EI(s, y, x) ((long)((y) + 2) * ((s)->nx + 4) + ((x) + 2))
#define LI(s, y, x) ((long)((y) + 1) * ((s)->nx + 2) + ((x) + 1))

/* Initial state: f* = f^eq(rho, 0) for the given density field. */
static void set_equilibrium_state(orc_sim* s, const double* rho) {
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            double feq[9];
            orc_equilibrium(rho[CI(s, y, x)], 0.0, 0.0, feq);
            for (int i = 0; i < 9; ++i) FI(s, s->f, i, y, x) = feq[i];
            s->rho[CI(s, y, x)] = rho[CI(s, y, x)];
            s->vx[CI(s, y, x)] = 0.0;
            s->vy[CI(s, y, x)] = 0.0;
        }
    s->step = 0;
    s->unstable_step = -1;
    s->hist_n = 0;
    s->int_peak_tau2 = 0.0;
    s->int_tau2 = 0.0;
    for (int w = 0; w < 2; ++w) {
        s->run[0][w] = -INFINITY;
        s->run[1][w] = INFINITY;
        s->run[2][w] = -INFINITY;
        s->run[3][w] = INFINITY;
    }
    memset(s->tau_w, 0, 2 * (size_t)s->nx * sizeof(double));
    memset(s->p_w, 0, 2 * (size_t)s->nx * sizeof(double));
}

int orc_init_density(orc_sim* s, const double* rho) {
    set_equilibrium_state(s, rho);
    return ORC_OK;
}

/* Liquid plug spanning the channel plus a wall film on both walls, the rest
   gas, at the Maxwell coexistence densities, with additive uniform noise of
   amplitude noise_amp drawn cell by cell (row-major) from SplitMix64(seed). */
int orc_init_plug(orc_sim* s, double plug_len, double film, double x_center,
                  double noise_amp, uint64_t seed) {
    if (isnan(s->rho_l)) return ORC_EINVAL;
    if (isnan(x_center)) x_center = s->nx / 4.0 + plug_len / 2.0;
    double* rho = (double*)malloc((size_t)s->nx * s->ny * sizeof(double));
    if (!rho) return ORC_ENOMEM;
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            int in_plug = (x >= x_center - plug_len / 2.0) && (x < x_center + plug_len / 2.0);
            int in_film = (y < film) || (y >= s->ny - film);
            double r = (in_plug || in_film) ? s->rho_l : s->rho_g;
            uint64_t z = orc_splitmix64(seed, (uint64_t)CI(s, y, x));
            double U = (double)(z >> 11) * (1.0 / 9007199254740992.0);
            rho[CI(s, y, x)] = r + noise_amp * (2.0 * U - 1.0);
        }
    set_equilibrium_state(s, rho);
    free(rho);
    return ORC_OK;
}

void orc_set_f(orc_sim* s, const double* f) {
    memcpy(s->f, f, 9 * sizeof(double) * s->nx * s->ny);
}

void orc_get_f(const orc_sim* s, double* f) {
    memcpy(f, s->f, 9 * sizeof(double) * s->nx * s->ny);
}

static int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

/* Stage 1: pull streaming, f_i(x) = f*_i(x - e_i), eq. 2.1 left-hand side. */
static void stage_stream(orc_sim* s) {
    int nx = s->nx, ny = s->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int i = 0; i < 9; ++i)
            for (int x = 0; x < nx; ++x) {
                int sx = x - EX[i], sy = y - EY[i];
                double v;
                if (!s->p.y_periodic && (sy < 0 || sy >= ny)) {
                    v = FI(s, s->f, OPP[i], y, x);            /* halfway bounce-back */
                } else {
                    if (s->p.y_periodic) sy = wrap(sy, ny);
                    if (sx < 0 || sx >= nx)
                        sx = s->p.x_periodic ? wrap(sx, nx) : (sx < 0 ? 0 : nx - 1);
                    v = FI(s, s->f, i, sy, sx);
                }
                FI(s, s->fs, i, y, x) = v;
            }
}

/* Stage 2: density and momentum. */
static void stage_moments(orc_sim* s) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int i = 0; i < 9; ++i) {
                double v = FI(s, s->fs, i, y, x);
                r += v;
                jx += v * EX[i];
                jy += v * EY[i];
            }
            s->rho[CI(s, y, x)] = r;
            s->jx[CI(s, y, x)] = jx;
            s->jy[CI(s, y, x)] = jy;
        }
}

/* Stage 3: density with a ghost ring of width 2, and the EOS field
   phi = k^2 p0(rho) - c_s^2 rho (the nonideal part of eq. 2.17). */
static void stage_ghosts_and_phi(orc_sim* s) {
    int nx = s->nx, ny = s->ny;
    double k2 = s->p.k * s->p.k;
#pragma omp parallel for schedule(static)
    for (int y = -2; y < ny + 2; ++y)
        for (int x = -2; x < nx + 2; ++x) {
            double r;
            if (y < 0 || y >= ny) {
                if (s->p.y_periodic) {
                    int yy = wrap(y, ny);
                    int xx = (x < 0 || x >= nx) ? (s->p.x_periodic ? wrap(x, nx) : (x < 0 ? 0 : nx - 1)) : x;
                    r = s->rho[CI(s, yy, xx)];
                } else {
                    r = s->rho_w;                              /* wetting wall */
                }
            } else if (x < 0 || x >= nx) {
                int xx = s->p.x_periodic ? wrap(x, nx) : (x < 0 ? 0 : nx - 1);
                r = s->rho[CI(s, y, xx)];
            } else {
                r = s->rho[CI(s, y, x)];
            }
            s->rext[EI(s, y, x)] = r;
            s->phiext[EI(s, y, x)] = k2 * eos_p(&s->eos, r, 0) - r / 3.0;
        }
}

/* Stage 4: Laplacian of the density on the grid plus one ghost ring. */
static void stage_laplacian(orc_sim* s) {
    long pitch = s->nx + 4;
#pragma omp parallel for schedule(static)
    for (int y = -1; y < s->ny + 1; ++y)
        for (int x = -1; x < s->nx + 1; ++x)
            s->lap[LI(s, y, x)] = lap_at(s->rext + EI(s, y, x), pitch);
}

/* Stage 5: the nonideal force of eq. 2.17 plus the driving body force. */
static void stage_force(orc_sim* s) {
    double g = s->p.dp / s->nx;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            double gpx, gpy, glx, gly;
            grad_at(s->phiext + EI(s, y, x), s->nx + 4, &gpx, &gpy);
            grad_at(s->lap + LI(s, y, x), s->nx + 2, &glx, &gly);
            double r = s->rho[CI(s, y, x)];
            s->Fx[CI(s, y, x)] = -gpx + s->p.kappa * r * glx + g;
            s->Fy[CI(s, y, x)] = -gpy + s->p.kappa * r * gly;
        }
}

/* Stage 6: velocities and MRT collision, writing the new post-collision state. */
static void stage_collide(orc_sim* s) {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < s->ny; ++y)
        for (int x = 0; x < s->nx; ++x) {
            double f[9], fo[9], r, vx, vy;
            for (int i = 0; i < 9; ++i) f[i] = FI(s, s->fs, i, y, x);
            collide(&s->col, f, s->Fx[CI(s, y, x)], s->Fy[CI(s, y, x)], fo, &r, &vx, &vy);
            for (int i = 0; i < 9; ++i) FI(s, s->f, i, y, x) = fo[i];
            s->vx[CI(s, y, x)] = vx;
            s->vy[CI(s, y, x)] = vy;
        }
}

/* Wall pressure at column x of fluid row y1 (the first row next to a wall):
   the isotropic part of the pressure tensor of eq. 2.8 in mesh units,
   k^2 p0(rho) - kappa rho lap(rho) - kappa/2 |grad rho|^2, with the same
   stencils as the force (ghost rows at the wall density). */
static double wall_pressure(const orc_sim* s, int y1, int x) {
    double k2 = s->p.k * s->p.k;
    double r = s->rho[CI(s, y1, x)];
    double gx, gy;
    grad_at(s->rext + EI(s, y1, x), s->nx + 4, &gx, &gy);
    double L = s->lap[LI(s, y1, x)];
    return k2 * eos_p(&s->eos, r, 0) - s->p.kappa * r * L - 0.5 * s->p.kappa * (gx * gx + gy * gy);
}

/* Stage 7: wall shear and pressure on the first fluid row of each wall, and
   the per-step summary (extremes, sum of squares, running time integrals). */
static void stage_wall_diagnostics(orc_sim* s) {
    if (s->p.y_periodic) return;
    int nx = s->nx, ny = s->ny;
    double nu = (s->p.tau - 0.5) / 3.0;
    orc_summary sm;
    memset(&sm, 0, sizeof sm);
    sm.step = s->step;
    double peak2 = 0.0, sum2 = 0.0;
    for (int w = 0; w < 2; ++w) {
        int y1 = (w == 0) ? 0 : ny - 1;          /* s = 1/2 from the wall */
        int y2 = (w == 0) ? 1 : ny - 2;          /* s = 3/2 from the wall */
        for (int x = 0; x < nx; ++x) {
            double r = s->rho[CI(s, y1, x)];
            double dvds = (9.0 * s->vx[CI(s, y1, x)] - s->vx[CI(s, y2, x)]) / 3.0;
            double tw = r * nu * dvds;
            double pw = wall_pressure(s, y1, x);
            s->tau_w[w * nx + x] = tw;
            s->p_w[w * nx + x] = pw;
            if (x == 0 || tw > sm.tau_max[w]) { sm.tau_max[w] = tw; sm.x_tau_max[w] = x; }
            if (x == 0 || tw < sm.tau_min[w]) { sm.tau_min[w] = tw; sm.x_tau_min[w] = x; }
            if (x == 0 || pw > sm.p_max[w]) { sm.p_max[w] = pw; sm.x_p_max[w] = x; }
            if (x == 0 || pw < sm.p_min[w]) { sm.p_min[w] = pw; sm.x_p_min[w] = x; }
            if (tw * tw > peak2) peak2 = tw * tw;
            sum2 += tw * tw;
        }
    }
    s->int_peak_tau2 += peak2;
    s->int_tau2 += sum2;
    for (int w = 0; w < 2; ++w) {
        s->run[0][w] = fmax(s->run[0][w], sm.tau_max[w]);
        s->run[1][w] = fmin(s->run[1][w], sm.tau_min[w]);
        s->run[2][w] = fmax(s->run[2][w], sm.p_max[w]);
        s->run[3][w] = fmin(s->run[3][w], sm.p_min[w]);
        sm.run_tau_max[w] = s->run[0][w];
        sm.run_tau_min[w] = s->run[1][w];
        sm.run_p_max[w] = s->run[2][w];
        sm.run_p_min[w] = s->run[3][w];
    }
    sm.sum_tau2 = sum2;
    sm.int_peak_tau2 = s->int_peak_tau2;
    sm.int_tau2 = s->int_tau2;
    if (s->hist_n == s->hist_cap) {
        int64_t cap = s->hist_cap ? 2 * s->hist_cap : 1024;
        orc_summary* h = (orc_summary*)realloc(s->hist, (size_t)cap * sizeof *h);
        if (!h) return;
        s->hist = h;
        s->hist_cap = cap;
    }
    s->hist[s->hist_n++] = sm;
}

static int stability_check(orc_sim* s) {
    long n = (long)s->nx * s->ny;
    for (long c = 0; c < n; ++c) {
        double r = s->rho[c], vx = s->vx[c], vy = s->vy[c];
        if (isnan(r) || isnan(vx) || isnan(vy) || sqrt(vx * vx + vy * vy) > s->p.v_limit)
            return 0;
    }
    return 1;
}

int orc_step(orc_sim* s, int64_t n) {
    for (int64_t t = 0; t < n; ++t) {
        s->step += 1;
        stage_stream(s);
        stage_moments(s);
        stage_ghosts_and_phi(s);
        stage_laplacian(s);
        stage_force(s);
        stage_collide(s);
        stage_wall_diagnostics(s);
        int at_check = (s->step % s->p.check_every == 0) || (t == n - 1);
        if (at_check && s->unstable_step < 0 && !stability_check(s)) {
            s->unstable_step = s->step;
            return ORC_EUNSTABLE;
        }
    }
    return ORC_OK;
}

int64_t orc_step_count(const orc_sim* s) { return s->step; }
int64_t orc_unstable_step(const orc_sim* s) { return s->unstable_step; }

void orc_fields(const orc_sim* s, double* rho, double* vx, double* vy) {
    size_t n = (size_t)s->nx * s->ny;
    if (rho) memcpy(rho, s->rho, n * sizeof(double));
    if (vx) memcpy(vx, s->vx, n * sizeof(double));
    if (vy) memcpy(vy, s->vy, n * sizeof(double));
}

void orc_force(const orc_sim* s, double* Fx, double* Fy) {
    size_t n = (size_t)s->nx * s->ny;
    if (Fx) memcpy(Fx, s->Fx, n * sizeof(double));
    if (Fy) memcpy(Fy, s->Fy, n * sizeof(double));
}

void orc_eval_force(orc_sim* s, const double* rho, double* Fx, double* Fy, double* p_bot, double* p_top) {
    int nx = s->nx, ny = s->ny;
    memcpy(s->rho, rho, (size_t)nx * ny * sizeof(double));
    stage_ghosts_and_phi(s);
    stage_laplacian(s);
    stage_force(s);
    if (Fx) memcpy(Fx, s->Fx, (size_t)nx * ny * sizeof(double));
    if (Fy) memcpy(Fy, s->Fy, (size_t)nx * ny * sizeof(double));
    for (int w = 0; w < 2 && !s->p.y_periodic; ++w) {
        double* out = w == 0 ? p_bot : p_top;
        if (!out) continue;
        for (int x = 0; x < nx; ++x) out[x] = wall_pressure(s, w == 0 ? 0 : ny - 1, x);
    }
}

void orc_wall(const orc_sim* s, double* tau_bot, double* tau_top, double* p_bot, double* p_top) {
    size_t nx = (size_t)s->nx;
    if (tau_bot) memcpy(tau_bot, s->tau_w, nx * sizeof(double));
    if (tau_top) memcpy(tau_top, s->tau_w + nx, nx * sizeof(double));
    if (p_bot) memcpy(p_bot, s->p_w, nx * sizeof(double));
    if (p_top) memcpy(p_top, s->p_w + nx, nx * sizeof(double));
}

int64_t orc_history(const orc_sim* s, orc_summary* buf, int64_t cap) {
    int64_t n = s->hist_n < cap ? s->hist_n : cap;
    if (n > 0) memcpy(buf, s->hist + (s->hist_n - n), (size_t)n * sizeof *buf);
    return n;
}

void orc_totals(const orc_sim* s, double* mass, double* momx, double* momy) {
    double m = 0.0, px = 0.0, py = 0.0;
    long n = (long)s->nx * s->ny;
    for (long c = 0; c < n; ++c) {
        m += s->rho[c];
        px += s->rho[c] * s->vx[c];
        py += s->rho[c] * s->vy[c];
    }
    *mass = m;
    *momx = px;
    *momy = py;
}

/* Plug interfaces on the channel centreline: the crossings of the midpoint
   density (rho_g + rho_l)/2, linearly interpolated; the rear is the upstream
   (smaller x) one.  Positions are NaN unless the centreline holds exactly one
   liquid run away from both ends.  liquid_columns counts the columns whose
   minimum density over y exceeds the midpoint (0 once the plug has ruptured). */
int orc_interface(const orc_sim* s, double* x_rear, double* x_front, int* liquid_columns) {
    int nx = s->nx, ny = s->ny;
    double mid = 0.5 * (s->rho_g + s->rho_l);
    double* c = (double*)malloc((size_t)nx * sizeof(double));
    if (!c) return ORC_ENOMEM;
    for (int x = 0; x < nx; ++x) {
        if (ny % 2 == 0)
            c[x] = 0.5 * (s->rho[CI(s, ny / 2 - 1, x)] + s->rho[CI(s, ny / 2, x)]);
        else
            c[x] = s->rho[CI(s, ny / 2, x)];
    }
    int runs = 0, start = -1, end = -1;
    for (int x = 0; x < nx; ++x) {
        int liq = c[x] > mid;
        int prev = x > 0 ? (c[x - 1] > mid) : 0;
        if (liq && !prev) { runs++; start = x; }
        if (liq) end = x;
    }
    *x_rear = NAN;
    *x_front = NAN;
    if (runs == 1 && start > 0 && end < nx - 1) {
        *x_rear = (start - 1) + (mid - c[start - 1]) / (c[start] - c[start - 1]);
        *x_front = end + (c[end] - mid) / (c[end] - c[end + 1]);
    }
    int cols = 0;
    for (int x = 0; x < nx; ++x) {
        double mn = s->rho[CI(s, 0, x)];
        for (int y = 1; y < ny; ++y)
            if (s->rho[CI(s, y, x)] < mn) mn = s->rho[CI(s, y, x)];
        if (mn > mid) cols++;
    }
    *liquid_columns = cols;
    free(c);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Liquid components (aerosol detection, Sec. 3.2-3.3).  A plain breadth-first
 * flood fill: cells are visited in row-major order, each unvisited liquid cell
 * seeds a new component (so components come out ordered by first cell), and
 * the fill walks the 4 or 8 neighbours, wrapping across periodic edges.
 * ------------------------------------------------------------------------- */

/* Offset d of a coordinate from a reference, moved to the nearest image
   (-n/2 <= d < n/2) when the direction is periodic. */
static double nearest_image(int d, int n, int periodic) {
    if (periodic) {
        while (d < -n / 2) d += n;
        while (d >= n - n / 2) d -= n;
    }
    return (double)d;
}

static double wrap_into(double v, int n) {
    double r = fmod(v, (double)n);
    return r < 0 ? r + n : r;
}

int64_t orc_components_field(const double* rho, int nx, int ny, int x_periodic, int y_periodic, double threshold,
                             double rho_g, int connectivity, orc_component* out, int64_t cap) {
    if (!rho || nx < 1 || ny < 1 || (connectivity != 4 && connectivity != 8) || cap < 0 || (cap > 0 && !out) ||
        isnan(threshold))
        return ORC_EINVAL;
    const long n = (long)nx * ny;
    unsigned char* seen = (unsigned char*)calloc((size_t)n, 1);
    long* queue = (long*)malloc((size_t)n * sizeof(long));
    if (!seen || !queue) {
        free(seen);
        free(queue);
        return ORC_ENOMEM;
    }
    static const int dx8[8] = {1, -1, 0, 0, 1, -1, -1, 1};
    static const int dy8[8] = {0, 0, 1, -1, 1, 1, -1, -1};
    int64_t count = 0;
    for (long seed = 0; seed < n; ++seed) {
        if (seen[seed] || !(rho[seed] > threshold)) continue;
        const int x0 = (int)(seed % nx), y0 = (int)(seed / nx);
        orc_component c;
        c.first_cell = seed;
        c.cells = 0;
        c.wall = 0;
        c.mass = 0.0;
        c.excess_mass = 0.0;
        double sx = 0.0, sy = 0.0;
        long head = 0, tail = 0;
        queue[tail++] = seed;
        seen[seed] = 1;
        while (head < tail) {
            const long cell = queue[head++];
            const int x = (int)(cell % nx), y = (int)(cell / nx);
            c.cells += 1;
            c.mass += rho[cell];
            c.excess_mass += rho[cell] - rho_g;
            sx += nearest_image(x - x0, nx, x_periodic);
            sy += nearest_image(y - y0, ny, y_periodic);
            if (!y_periodic && (y == 0 || y == ny - 1)) c.wall = 1;
            for (int k = 0; k < connectivity; ++k) {
                int xn = x + dx8[k], yn = y + dy8[k];
                if (xn < 0 || xn >= nx) {
                    if (!x_periodic) continue;
                    xn = (xn + nx) % nx;
                }
                if (yn < 0 || yn >= ny) {
                    if (!y_periodic) continue;
                    yn = (yn + ny) % ny;
                }
                const long nb = (long)yn * nx + xn;
                if (!seen[nb] && rho[nb] > threshold) {
                    seen[nb] = 1;
                    queue[tail++] = nb;
                }
            }
        }
        c.cx = x_periodic ? wrap_into(x0 + sx / c.cells, nx) : x0 + sx / c.cells;
        c.cy = y_periodic ? wrap_into(y0 + sy / c.cells, ny) : y0 + sy / c.cells;
        if (count < cap) out[count] = c;
        count += 1;
    }
    free(seen);
    free(queue);
    return count;
}

int64_t orc_components(const orc_sim* s, double threshold, int connectivity, orc_component* out, int64_t cap) {
    if (isnan(threshold)) threshold = 0.5 * (s->rho_g + s->rho_l);
    if (isnan(threshold)) return ORC_EINVAL;
    return orc_components_field(s->rho, s->nx, s->ny, s->p.x_periodic, s->p.y_periodic, threshold, s->rho_g,
                                connectivity, out, cap);
}
