/*
 * at_oracle.c -- plain serial FP64 reference of the asynchrony-tolerant RK step.
 * TEST INFRASTRUCTURE ONLY (see at_oracle.h).  Written for readability, not
 * speed: whole-field arrays, one straight loop per formula, fixed summation
 * order, no blocking or fusion.  Compile with -ffp-contract=off.
 *
 * Algorithm of one step n -> n+1 (Sec. 2.3 of the paper, with the reading of
 * the multi-stage AT procedure stated there: every RK stage at PE-boundary and
 * buffer points is computed locally, and at old time levels those stages come
 * from the standard synchronous scheme):
 *
 *   cache  G[m][s]   synchronous stage s of the global level m:
 *                    G[m][0] = u^m,  G[m][s] = u^m + dt sum_{i<s} a_si Rsync(G[m][i])
 *   delays k~(p, side) per PE per step; effective k = clamp to the held history
 *   stage  V(s) = u^n + dt sum_{i<s} a_si K_i
 *          K_s at PE p's own points = R applied to the extended array:
 *              own points   g(V(s))
 *              halo points  sum_{l<J} w_l(k) g(G[n-k-l][s])   (zero weights skipped)
 *          g = the differentiated quantities (u itself for linear problems, the
 *              fluxes and primitives for nonlinear ones: fluxes are evaluated
 *              on each stored level, then extrapolated, Sec. 6)
 *   update u^{n+1} = u^n + dt sum_s b_s K_s, then fill G[n+1][*].
 */
#include "at_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXF 4
#define MAXQ 8
#define MAXS 4
#define MAXJ 8

/* ------------------------------------------------------------------------- */
/* Runge-Kutta tableaus in Butcher form (eq. rk1).                            */
/* ------------------------------------------------------------------------- */
typedef struct { int S; double a[MAXS][MAXS]; double b[MAXS]; } tableau;

static int get_tableau(int rk, tableau* t) {
    memset(t, 0, sizeof(*t));
    switch (rk) {
    case ORC_FE:       /* forward Euler                                        */
        t->S = 1; t->b[0] = 1.0; return 0;
    case ORC_RK2:      /* two-stage second order of eq. rk2 (Heun)              */
        t->S = 2; t->a[1][0] = 1.0; t->b[0] = 0.5; t->b[1] = 0.5; return 0;
    case ORC_SSPRK3:   /* three-stage third order (Shu-Osher SSP), "RK-3"       */
        t->S = 3; t->a[1][0] = 1.0; t->a[2][0] = 0.25; t->a[2][1] = 0.25;
        t->b[0] = 1.0 / 6.0; t->b[1] = 1.0 / 6.0; t->b[2] = 2.0 / 3.0; return 0;
    case ORC_RK4:      /* classical four-stage fourth order                      */
        t->S = 4; t->a[1][0] = 0.5; t->a[2][1] = 0.5; t->a[3][2] = 1.0;
        t->b[0] = 1.0 / 6.0; t->b[1] = 1.0 / 3.0; t->b[2] = 1.0 / 3.0; t->b[3] = 1.0 / 6.0;
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Central finite differences (standard textbook coefficients).              */
/*   d/dx    = (1/dx)   sum_o c1[o] (g[e+o] - g[e-o])                        */
/*   d2/dx2  = (1/dx^2) (c2[0] g[e] + sum_o c2[o] (g[e+o] + g[e-o]))         */
/* ------------------------------------------------------------------------- */
static const double FD2_C1[2] = {0.0, 0.5};
static const double FD2_C2[2] = {-2.0, 1.0};
static const double FD4_C1[3] = {0.0, 2.0 / 3.0, -1.0 / 12.0};
static const double FD4_C2[3] = {-5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0};
static const double FD8_C1[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};
static const double FD8_C2[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

int orc_halo_width(int scheme) {
    switch (scheme) {
    case ORC_FD2: return 1;
    case ORC_FD4: return 2;
    case ORC_FD8: return 4;
    case ORC_WENO5: case ORC_WENO5I: return 3;
    }
    return -1;
}

/* Number of time levels the AT halo extrapolation uses (Table A: 3 levels for
 * the 4th-order schemes; eqs. atRecon/beta2AT*: 2 levels for AT-WENO; eq. at1:
 * 2 levels for 2nd order).  The 8th-order interior takes Table A's 3 levels at
 * PE boundaries: 5 levels (the same family one order up) is selectable through
 * at_levels but unstable for delays >= 1 at any practical CFL number. */
int orc_levels(int scheme, int mode, int at_levels) {
    if (mode != ORC_AT) return 1;
    if (at_levels > 0) return at_levels;
    switch (scheme) {
    case ORC_FD2: return 2;
    case ORC_FD4: return 3;
    case ORC_FD8: return 3;
    case ORC_WENO5: case ORC_WENO5I: return 2;
    }
    return -1;
}

int orc_nfields(int pde) {
    switch (pde) {
    case ORC_PDE_ADV_DIFF: case ORC_PDE_ADR_LOGISTIC: case ORC_PDE_BURGERS: return 1;
    case ORC_PDE_EULER: return 3;
    case ORC_PDE_REACTIVE_EULER: case ORC_PDE_REACTIVE_NS: return 4;
    }
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Lagrange extrapolation in time: levels t_l = -(k + l), l = 0..J-1, to t=0: */
/*   w_l = prod_{m != l} (0 - t_m) / (t_l - t_m) = prod_{m != l} (k+m)/(m-l)  */
/* ------------------------------------------------------------------------- */
int orc_extrap_weights(int J, int k, double* w) {
    if (J < 1 || J > MAXJ || k < 0) return ORC_EINVAL;
    for (int l = 0; l < J; ++l) {
        double num = 1.0, den = 1.0;
        for (int m = 0; m < J; ++m) {
            if (m == l) continue;
            num *= (double)(k + m);
            den *= (double)(m - l);
        }
        w[l] = num / den;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Delay draws: SplitMix64 finaliser as a counter-based hash.                 */
/* ------------------------------------------------------------------------- */
static const uint64_t GOLDEN = 0x9e3779b97f4a7c15ULL;

uint64_t orc_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

int orc_draw(const orc_problem* pb, int64_t step, int64_t idx, int side) {
    uint64_t z = orc_mix64(pb->seed + GOLDEN * (uint64_t)(pb->problem_id + 1));
    z = orc_mix64(z + GOLDEN * (uint64_t)(step + 1));
    z = orc_mix64(z + GOLDEN * (uint64_t)(2 * idx + side + 1));
    uint64_t u32 = z >> 32;
    if (pb->n_cdf == 0)
        return (int)((u32 * (uint64_t)(pb->kmax + 1)) >> 32);
    int k = 0;
    while (k < pb->kmax && u32 >= pb->cdf[k]) ++k;
    return k;
}

/* ------------------------------------------------------------------------- */
/* Physics: differentiated quantities, wave speed, source.                   */
/* ------------------------------------------------------------------------- */
static int is_weno(const orc_problem* pb) { return pb->scheme == ORC_WENO5 || pb->scheme == ORC_WENO5I; }

static int nquant(const orc_problem* pb) {
    int F = orc_nfields(pb->pde);
    if (is_weno(pb)) return 2 * F;                 /* Q_f then C_f             */
    if (pb->pde == ORC_PDE_REACTIVE_NS)            /* C1..C4, u, T, Y (flux)   */
        return pb->form == 1 ? 5 : 7;              /* rho, u, p, T, Y (chain)  */
    return 1;                                      /* u                        */
}

/* Reacting gas with one-step chemistry, R = 1:  E = T/(gamma-1) + u^2/2 + qY. */
static void reactive_primitives(const orc_problem* pb, const double* q,
                                double* rho, double* u, double* T, double* Y) {
    *rho = q[0];
    *u = q[1] / q[0];
    double E = q[2] / q[0];
    *Y = q[3] / q[0];
    *T = (pb->gamma - 1.0) * (E - 0.5 * (*u) * (*u) - pb->q * (*Y));
}

/* convective flux vector C(Q) of eq. convEq (one-step-chemistry form) */
static void conv_flux(const orc_problem* pb, const double* q, double* C) {
    switch (pb->pde) {
    case ORC_PDE_ADV_DIFF: case ORC_PDE_ADR_LOGISTIC:
        C[0] = pb->c * q[0]; return;
    case ORC_PDE_BURGERS:
        C[0] = 0.5 * q[0] * q[0]; return;
    case ORC_PDE_EULER: {
        double u = q[1] / q[0];
        double p = (pb->gamma - 1.0) * (q[2] - 0.5 * q[1] * u);
        C[0] = q[1]; C[1] = q[1] * u + p; C[2] = u * (q[2] + p); return;
    }
    case ORC_PDE_REACTIVE_EULER: case ORC_PDE_REACTIVE_NS: {
        double rho, u, T, Y;
        reactive_primitives(pb, q, &rho, &u, &T, &Y);
        double p = rho * T;
        C[0] = q[1]; C[1] = q[1] * u + p; C[2] = u * (q[2] + p); C[3] = q[3] * u; return;
    }
    }
}

static void quantities(const orc_problem* pb, const double* q, double* g) {
    int F = orc_nfields(pb->pde);
    if (is_weno(pb)) {
        double C[MAXF];
        conv_flux(pb, q, C);
        for (int f = 0; f < F; ++f) { g[f] = q[f]; g[F + f] = C[f]; }
        return;
    }
    if (pb->pde == ORC_PDE_REACTIVE_NS) {
        double C[MAXF], rho, u, T, Y;
        reactive_primitives(pb, q, &rho, &u, &T, &Y);
        if (pb->form == 1) {
            g[0] = rho; g[1] = u; g[2] = rho * T; g[3] = T; g[4] = Y;
            return;
        }
        conv_flux(pb, q, C);
        g[0] = C[0]; g[1] = C[1]; g[2] = C[2]; g[3] = C[3]; g[4] = u; g[5] = T; g[6] = Y;
        return;
    }
    g[0] = q[0];
}

/* maximum local wave speed |u| + c (Sec. 3, after eq. Csplit) */
static double wave_speed(const orc_problem* pb, const double* q) {
    switch (pb->pde) {
    case ORC_PDE_ADV_DIFF: case ORC_PDE_ADR_LOGISTIC: return fabs(pb->c);
    case ORC_PDE_BURGERS: return fabs(q[0]);
    case ORC_PDE_EULER: {
        double u = q[1] / q[0];
        double p = (pb->gamma - 1.0) * (q[2] - 0.5 * q[1] * u);
        return fabs(u) + sqrt(pb->gamma * p / q[0]);
    }
    case ORC_PDE_REACTIVE_EULER: case ORC_PDE_REACTIVE_NS: {
        double rho, u, T, Y;
        reactive_primitives(pb, q, &rho, &u, &T, &Y);
        return fabs(u) + sqrt(pb->gamma * T);
    }
    }
    return 0.0;
}

/* one-step Arrhenius rate of fuel consumption: omega = -B rho Y exp(-Ea/T) */
static double arrhenius(const orc_problem* pb, const double* q) {
    double rho, u, T, Y;
    reactive_primitives(pb, q, &rho, &u, &T, &Y);
    return -pb->b * rho * Y * exp(-pb->ea / T);
}

/* ------------------------------------------------------------------------- */
/* WENO5-JS reconstruction at the right edge of v2 from v0..v4 (eqs. interpS  */
/* reconstruction form atRecon at zero delay, betaS, omg, idRec).            */
/* ------------------------------------------------------------------------- */
static double weno5(double eps, double v0, double v1, double v2, double v3, double v4) {
    double p0 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) / 6.0;
    double p1 = (-v1 + 5.0 * v2 + 2.0 * v3) / 6.0;
    double p2 = (2.0 * v2 + 5.0 * v3 - v4) / 6.0;
    double b0 = 13.0 / 12.0 * (v0 - 2.0 * v1 + v2) * (v0 - 2.0 * v1 + v2)
              + 0.25 * (v0 - 4.0 * v1 + 3.0 * v2) * (v0 - 4.0 * v1 + 3.0 * v2);
    double b1 = 13.0 / 12.0 * (v1 - 2.0 * v2 + v3) * (v1 - 2.0 * v2 + v3)
              + 0.25 * (v1 - v3) * (v1 - v3);
    double b2 = 13.0 / 12.0 * (v2 - 2.0 * v3 + v4) * (v2 - 2.0 * v3 + v4)
              + 0.25 * (3.0 * v2 - 4.0 * v3 + v4) * (3.0 * v2 - 4.0 * v3 + v4);
    double a0 = 0.1 / ((eps + b0) * (eps + b0));
    double a1 = 0.6 / ((eps + b1) * (eps + b1));
    double a2 = 0.3 / ((eps + b2) * (eps + b2));
    return (a0 * p0 + a1 * p1 + a2 * p2) / (a0 + a1 + a2);
}

/* ------------------------------------------------------------------------- */
/* WENO5 in interpolation form: the value at the right edge of v2 from the   */
/* point values v0..v4 (eq. interpS: quadratic interpolants of the three     */
/* three-point candidates evaluated half a cell right of v2; eq. betaS:      */
/* smoothness indicators, those of eq. bet1 for the candidate polynomials;   */
/* eq. omg with the ideal weights 1/16, 5/8, 5/16 of eq. fullSten).          */
/* ------------------------------------------------------------------------- */
static double weno5i(double eps, double v0, double v1, double v2, double v3, double v4, double* beta) {
    double p0 = 3.0 / 8.0 * v0 - 5.0 / 4.0 * v1 + 15.0 / 8.0 * v2;
    double p1 = -1.0 / 8.0 * v1 + 3.0 / 4.0 * v2 + 3.0 / 8.0 * v3;
    double p2 = 3.0 / 8.0 * v2 + 3.0 / 4.0 * v3 - 1.0 / 8.0 * v4;
    /* eq. betaS: the quadratic forms of eq. bet1 for the three candidates, evaluated as
     * 13/12 (second difference)^2 + 1/4 (first difference)^2, the same forms as the
     * printed expansion (which loses the small indicators of smooth data to cancellation
     * when the values are large) */
    double b0 = 13.0 / 12.0 * (v0 - 2.0 * v1 + v2) * (v0 - 2.0 * v1 + v2)
              + 0.25 * (v0 - 4.0 * v1 + 3.0 * v2) * (v0 - 4.0 * v1 + 3.0 * v2);
    double b1 = 13.0 / 12.0 * (v1 - 2.0 * v2 + v3) * (v1 - 2.0 * v2 + v3)
              + 0.25 * (v1 - v3) * (v1 - v3);
    double b2 = 13.0 / 12.0 * (v2 - 2.0 * v3 + v4) * (v2 - 2.0 * v3 + v4)
              + 0.25 * (3.0 * v2 - 4.0 * v3 + v4) * (3.0 * v2 - 4.0 * v3 + v4);
    double a0 = (1.0 / 16.0) / ((eps + b0) * (eps + b0));
    double a1 = (5.0 / 8.0) / ((eps + b1) * (eps + b1));
    double a2 = (5.0 / 16.0) / ((eps + b2) * (eps + b2));
    if (beta) {
        beta[0] = b0;
        beta[1] = b1;
        beta[2] = b2;
    }
    return (a0 * p0 + a1 * p1 + a2 * p2) / (a0 + a1 + a2);
}

double orc_weno_interp(double eps, const double* v, double* beta) {
    return weno5i(eps, v[0], v[1], v[2], v[3], v[4], beta);
}

/* ------------------------------------------------------------------------- */
/* Right-hand side on an extended array.                                     */
/*   np own points at extended index e = H + j, j in [0, np)                 */
/*   g[k][e]  differentiated quantities, e in [0, np + 2H)                   */
/*   lam[e]   wave speed (WENO only)                                         */
/*   vown[f][j] own state (for sources and primitives)                        */
/*   K[f][j]  output                                                         */
/*   flux     optional (np + 1) x F interface fluxes (WENO)                  */
/* ------------------------------------------------------------------------- */
static void fd_coefs(int scheme, const double** c1, const double** c2) {
    switch (scheme) {
    case ORC_FD2: *c1 = FD2_C1; *c2 = FD2_C2; return;
    case ORC_FD4: *c1 = FD4_C1; *c2 = FD4_C2; return;
    default:      *c1 = FD8_C1; *c2 = FD8_C2; return;
    }
}

static double d1(const double* g, int e, int H, const double* c1, double dx) {
    double s = 0.0;
    for (int o = 1; o <= H; ++o) s += c1[o] * (g[e + o] - g[e - o]);
    return s / dx;
}

static double d2(const double* g, int e, int H, const double* c2, double dx) {
    double s = c2[0] * g[e];
    for (int o = 1; o <= H; ++o) s += c2[o] * (g[e + o] + g[e - o]);
    return s / (dx * dx);
}

/* ------------------------------------------------------------------------- */
/* Non-periodic ends (bc = 1).                                                */
/* Convective terms at an end point in characteristic form (LODI relations of */
/* Thompson 1987 / Poinsot & Lele 1992, for the one-step-chemistry gas):      */
/*   L1 = (u - c)(p_x - rho c u_x)    speed u - c                             */
/*   L2 = u (c^2 rho_x - p_x)         speed u                                 */
/*   L3 = u Y_x                       speed u                                 */
/*   L5 = (u + c)(p_x + rho c u_x)    speed u + c                             */
/* A wave entering the domain (speed > 0 at the left end, < 0 at the right)   */
/* has its amplitude set to zero (non-reflecting).  With                      */
/*   d1 = (L2 + (L5 + L1)/2) / c^2,  d2 = (L5 + L1)/2,  d3 = (L5 - L1)/(2 rho c)*/
/* the time derivatives are rho_t = -d1, u_t = -d3, p_t = -d2, Y_t = -L3, and  */
/* for the conserved state (rho E = p/(gamma-1) + rho u^2/2 + q rho Y):       */
/*   (rho)_t   = -d1                                                          */
/*   (rho u)_t = -(u d1 + rho d3)                                             */
/*   (rho Y)_t = -(Y d1 + rho L3)                                             */
/*   (rho E)_t = -(u^2 d1 / 2 + d2/(gamma-1) + rho u d3) + q (rho Y)_t        */
/* side: 0 left end, 1 right end; drop = 0 keeps every wave (the full         */
/* convective derivative, for the pins).                                     */
/* ------------------------------------------------------------------------- */
int orc_lodi(const orc_problem* pb, int side, int drop, const double* prim, const double* dprim,
             double* out) {
    const double rho = prim[0], u = prim[1], p = prim[2], Y = prim[3];
    const double rx = dprim[0], ux = dprim[1], px = dprim[2], Yx = dprim[3];
    const double gm = pb->gamma;
    const double c = sqrt(gm * p / rho);
    double L1 = (u - c) * (px - rho * c * ux);
    double L2 = u * (c * c * rx - px);
    double L3 = u * Yx;
    double L5 = (u + c) * (px + rho * c * ux);
    if (drop) {
        /* incoming: positive speed at the left end, negative at the right end */
        const double sgn = side == 0 ? 1.0 : -1.0;
        if (sgn * (u - c) > 0.0) L1 = 0.0;
        if (sgn * u > 0.0) { L2 = 0.0; L3 = 0.0; }
        if (sgn * (u + c) > 0.0) L5 = 0.0;
    }
    const double d1 = (L2 + 0.5 * (L5 + L1)) / (c * c);
    const double d2 = 0.5 * (L5 + L1);
    const double d3 = (L5 - L1) / (2.0 * rho * c);
    out[0] = -d1;
    out[1] = -(u * d1 + rho * d3);
    out[3] = -(Y * d1 + rho * L3);
    out[2] = -(0.5 * u * u * d1 + d2 / (gm - 1.0) + rho * u * d3) + pb->q * out[3];
    return ORC_OK;
}

/* primitives (rho, u, p, T, Y) at ext position e from the reactive NS quantities
 * C1 = rho u, C2 = rho u^2 + p, u, T, Y (g[0], g[1], g[4], g[5], g[6]) */
static void rns_prims_at(double** g, int e, double* rho, double* u, double* p, double* T, double* Y) {
    *u = g[4][e];
    *T = g[5][e];
    *Y = g[6][e];
    *p = g[1][e] - g[0][e] * (*u);
    *rho = *p / *T;
}

/* reactive NS right-hand side at a point whose stencil would leave the domain
 * (bc = 1): own point j at ext position e, global index x. */
static void rns_end_rhs(const orc_problem* pb, double** g, int e, int64_t x, const double* q,
                        double* Kq) {
    const int64_t N = pb->n;
    const double dx = pb->lx / (double)N;
    const double gm = pb->gamma;
    const double kappa = pb->mu * gm / ((gm - 1.0) * pb->pr);
    const double rhoD = pb->mu / (pb->pr * pb->le);
    double rho, u, p, T, Y;
    rns_prims_at(g, e, &rho, &u, &p, &T, &Y);
    double ux, uxx, Txx, Yxx, conv[4];
    if (x == 0 || x == N - 1) {
        /* second-order one-sided differences, inward direction sg */
        const int sg = x == 0 ? 1 : -1;
        double f[4][5];   /* points e, e+sg, e+2sg, e+3sg: rho, u, p, T, Y */
        for (int m = 0; m < 4; ++m)
            rns_prims_at(g, e + sg * m, &f[m][0], &f[m][1], &f[m][2], &f[m][3], &f[m][4]);
        double d1v[5], d2v[5];
        for (int v = 0; v < 5; ++v) {
            d1v[v] = (double)sg * (-3.0 * f[0][v] + 4.0 * f[1][v] - f[2][v]) / (2.0 * dx);
            d2v[v] = (2.0 * f[0][v] - 5.0 * f[1][v] + 4.0 * f[2][v] - f[3][v]) / (dx * dx);
        }
        const double prim[4] = {rho, u, p, Y};
        const double dprim[4] = {d1v[0], d1v[1], d1v[2], d1v[4]};
        orc_lodi(pb, x == 0 ? 0 : 1, 1, prim, dprim, conv);
        ux = d1v[1];
        uxx = d2v[1];
        Txx = d2v[3];
        Yxx = d2v[4];
    } else {
        /* second-order central differences of the conservative fluxes */
        for (int f = 0; f < 4; ++f) conv[f] = -(g[f][e + 1] - g[f][e - 1]) / (2.0 * dx);
        ux = (g[4][e + 1] - g[4][e - 1]) / (2.0 * dx);
        uxx = (g[4][e + 1] - 2.0 * g[4][e] + g[4][e - 1]) / (dx * dx);
        Txx = (g[5][e + 1] - 2.0 * g[5][e] + g[5][e - 1]) / (dx * dx);
        Yxx = (g[6][e + 1] - 2.0 * g[6][e] + g[6][e - 1]) / (dx * dx);
    }
    Kq[0] = conv[0];
    Kq[1] = conv[1] + (4.0 / 3.0) * pb->mu * uxx;
    Kq[2] = conv[2] + (4.0 / 3.0) * pb->mu * (ux * ux + u * uxx) + kappa * Txx + pb->q * rhoD * Yxx;
    Kq[3] = conv[3] + rhoD * Yxx + arrhenius(pb, q);
}

/* lo: global index of own point 0 (for the non-periodic ends) */
static void rhs_region(const orc_problem* pb, int64_t lo, int64_t np, double** g, const double* lam,
                       double** vown, double** K, double* flux) {
    const int F = orc_nfields(pb->pde);
    const int H = orc_halo_width(pb->scheme);
    const double dx = pb->lx / (double)pb->n;

    if (is_weno(pb)) {
        /* local Lax-Friedrichs splitting C+- = (C +- alpha Q)/2 with alpha the
         * larger wave speed of the two points beside the interface (eq. Csplit),
         * WENO5 for C+ (left-biased) and C- (right-biased), flux difference
         * (eq. wender). */
        double* Fi = (double*)malloc(sizeof(double) * (size_t)(np + 1) * F);
        for (int64_t ii = 0; ii <= np; ++ii) {
            int64_t i = ii + H - 1;            /* interface between e=i and e=i+1 */
            double al = lam[i] > lam[i + 1] ? lam[i] : lam[i + 1];
            for (int f = 0; f < F; ++f) {
                const double* Q = g[f];
                const double* C = g[F + f];
                double fp[5], fm[5];
                for (int m = 0; m < 5; ++m) {
                    fp[m] = 0.5 * (C[i - 2 + m] + al * Q[i - 2 + m]);
                    fm[m] = 0.5 * (C[i + 3 - m] - al * Q[i + 3 - m]);
                }
                double Fp, Fm;
                if (pb->scheme == ORC_WENO5I) {     /* interpolation form */
                    Fp = weno5i(pb->weno_eps, fp[0], fp[1], fp[2], fp[3], fp[4], NULL);
                    Fm = weno5i(pb->weno_eps, fm[0], fm[1], fm[2], fm[3], fm[4], NULL);
                } else {
                    Fp = weno5(pb->weno_eps, fp[0], fp[1], fp[2], fp[3], fp[4]);
                    Fm = weno5(pb->weno_eps, fm[0], fm[1], fm[2], fm[3], fm[4]);
                }
                Fi[ii * F + f] = Fp + Fm;
            }
        }
        for (int64_t j = 0; j < np; ++j) {
            double q[MAXF];
            for (int f = 0; f < F; ++f) q[f] = vown[f][j];
            for (int f = 0; f < F; ++f)
                K[f][j] = -(Fi[(j + 1) * F + f] - Fi[j * F + f]) / dx;
            if (pb->pde == ORC_PDE_REACTIVE_EULER) K[3][j] += arrhenius(pb, q);
            if (pb->pde == ORC_PDE_ADR_LOGISTIC) K[0][j] += pb->r * q[0] * (1.0 - q[0]);
        }
        if (flux) memcpy(flux, Fi, sizeof(double) * (size_t)(np + 1) * F);
        free(Fi);
        return;
    }

    const double *c1, *c2;
    fd_coefs(pb->scheme, &c1, &c2);
    if (pb->pde == ORC_PDE_REACTIVE_NS) {
        /* one-step-chemistry Navier-Stokes (eq. ge with constant mu, Pr, Le):
         * tau = 4/3 mu u_x, heat flux -kappa T_x - q rhoD Y_x, J = -rhoD Y_x */
        const double gm = pb->gamma;
        const double kappa = pb->mu * gm / ((gm - 1.0) * pb->pr);
        const double rhoD = pb->mu / (pb->pr * pb->le);
        for (int64_t j = 0; j < np; ++j) {
            int e = (int)(j + H);
            double q[MAXF];
            for (int f = 0; f < F; ++f) q[f] = vown[f][j];
            const int64_t x = lo + j;
            if (pb->bc == 1 && (x < H || x >= pb->n - H)) {
                double Kq[4];
                rns_end_rhs(pb, g, e, x, q, Kq);
                for (int f = 0; f < 4; ++f) K[f][j] = Kq[f];
                continue;
            }
            double rho, u, T, Y;
            reactive_primitives(pb, q, &rho, &u, &T, &Y);
            double dC0, dC1, dC2, dC3, ux, uxx, Txx, Yxx;
            if (pb->form == 1) {
                /* chain rule: the convective products differentiated through the
                 * primitives, e.g. (rho u Y)_x = rho u Y_x + rho u_x Y + rho_x u Y */
                const double p = rho * T;
                double rx = d1(g[0], e, H, c1, dx), px = d1(g[2], e, H, c1, dx);
                double Yx = d1(g[4], e, H, c1, dx);
                ux = d1(g[1], e, H, c1, dx);
                uxx = d2(g[1], e, H, c2, dx);
                Txx = d2(g[3], e, H, c2, dx);
                Yxx = d2(g[4], e, H, c2, dx);
                /* rho E = p/(gamma-1) + rho u^2/2 + q rho Y */
                double dE = px / (gm - 1.0) + 0.5 * rx * u * u + rho * u * ux + pb->q * (rx * Y + rho * Yx);
                dC0 = rx * u + rho * ux;
                dC1 = rx * u * u + 2.0 * rho * u * ux + px;
                dC2 = ux * (q[2] + p) + u * (dE + px);
                dC3 = rho * u * Yx + rho * ux * Y + rx * u * Y;
            } else {
                dC0 = d1(g[0], e, H, c1, dx);
                dC1 = d1(g[1], e, H, c1, dx);
                dC2 = d1(g[2], e, H, c1, dx);
                dC3 = d1(g[3], e, H, c1, dx);
                ux = d1(g[4], e, H, c1, dx);
                uxx = d2(g[4], e, H, c2, dx);
                Txx = d2(g[5], e, H, c2, dx);
                Yxx = d2(g[6], e, H, c2, dx);
            }
            K[0][j] = -dC0;
            K[1][j] = -dC1 + (4.0 / 3.0) * pb->mu * uxx;
            K[2][j] = -dC2 + (4.0 / 3.0) * pb->mu * (ux * ux + u * uxx) + kappa * Txx
                      + pb->q * rhoD * Yxx;
            K[3][j] = -dC3 + rhoD * Yxx + arrhenius(pb, q);
        }
        return;
    }
    /* advection-diffusion(-logistic): u_t = -c u_x + alpha u_xx (+ r u (1-u)) */
    for (int64_t j = 0; j < np; ++j) {
        int e = (int)(j + H);
        double k = -pb->c * d1(g[0], e, H, c1, dx) + pb->alpha * d2(g[0], e, H, c2, dx);
        if (pb->pde == ORC_PDE_ADR_LOGISTIC) {
            double u = vown[0][j];
            k += pb->r * u * (1.0 - u);
        }
        K[0][j] = k;
    }
}

/* ------------------------------------------------------------------------- */
/* Validation                                                                */
/* ------------------------------------------------------------------------- */
static int validate(const orc_problem* pb) {
    if (orc_nfields(pb->pde) < 0 || orc_halo_width(pb->scheme) < 0) return ORC_EINVAL;
    if (pb->mode < ORC_SYNC || pb->mode > ORC_AT) return ORC_EINVAL;
    tableau t;
    if (get_tableau(pb->rk, &t)) return ORC_EINVAL;
    if (pb->granularity < ORC_PER_PE || pb->granularity > ORC_PER_BOUNDARY) return ORC_EINVAL;
    if (pb->n < 1 || pb->p < 1 || pb->p > pb->n) return ORC_EINVAL;
    if (pb->kmax < 0 || pb->kmax > 15) return ORC_EINVAL;
    if (pb->n_cdf != 0 && pb->n_cdf != pb->kmax) return ORC_EINVAL;
    if (pb->at_levels < 0 || pb->at_levels > MAXJ) return ORC_EINVAL;
    if (!(pb->dt > 0.0) || !(pb->lx > 0.0)) return ORC_EINVAL;
    int weno = is_weno(pb);
    switch (pb->pde) {
    case ORC_PDE_ADV_DIFF: case ORC_PDE_ADR_LOGISTIC:
        if (weno && pb->alpha != 0.0) return ORC_EINVAL;
        break;
    case ORC_PDE_BURGERS: case ORC_PDE_EULER: case ORC_PDE_REACTIVE_EULER:
        if (!weno) return ORC_EINVAL;
        break;
    case ORC_PDE_REACTIVE_NS:
        if (weno) return ORC_EINVAL;
        break;
    }
    if (pb->bc != 0 && pb->bc != 1) return ORC_EINVAL;
    /* the chain-rule form: reactive NS with periodic ends */
    if (pb->form != 0 && pb->form != 1) return ORC_EINVAL;
    if (pb->form == 1 && (pb->pde != ORC_PDE_REACTIVE_NS || pb->bc != 0)) return ORC_EINVAL;
    if (pb->bc == 1) {
        /* the end closure reads four points inside the first and the last PE */
        if (pb->pde != ORC_PDE_REACTIVE_NS) return ORC_EINVAL;
        if ((1 * pb->n) / pb->p < 4 || pb->n - ((int64_t)(pb->p - 1) * pb->n) / pb->p < 4) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Run state                                                                 */
/* ------------------------------------------------------------------------- */
struct orc_run {
    orc_problem pb;
    tableau tb;
    int F, H, J, D, S, nq;
    int64_t N, n;
    double* G;        /* D x S x F x N : synchronous stages of held levels     */
    double* K;        /* S x F x N     : stage right-hand sides                */
    double* V;        /* F x N         : current stage state                   */
    double* unew;     /* F x N                                                   */
    double* Rg;       /* S x F x N     : Rsync of cached stages                 */
    double* ext;      /* (nq + 1) x (N + 2H) extended arrays (+ wave speed)      */
    double* flux;     /* (N + P) x F   : interface fluxes of the last AT RHS     */
    int* keff;        /* P x 2                                                   */
    /* delay log: step-major, P x 2 per step */
    int64_t log_n, log_cap;
    uint8_t *drawn, *eff;
    /* override */
    int64_t ov_step0, ov_n;
    uint8_t* ov;
};

static double* Gptr(const orc_run* r, int64_t m, int s) {
    int64_t slot = ((m % r->D) + r->D) % r->D;
    return r->G + ((slot * r->S + s) * (int64_t)r->F) * r->N;
}

static int64_t pe_lo(const orc_run* r, int64_t p) { return (p * r->N) / r->pb.p; }

static int64_t wrap(int64_t x, int64_t N) { return ((x % N) + N) % N; }

/* out = u + dt * sum_{i<s} arow[i] K_i  (i ascending); s == 0 gives u.     */
static void stage_combine(const orc_run* r, const double* u, const double* Kbase,
                          const double* arow, int s, double* out) {
    const int64_t FN = (int64_t)r->F * r->N;
    if (s == 0) { memcpy(out, u, sizeof(double) * (size_t)FN); return; }
    for (int64_t i = 0; i < FN; ++i) {
        double acc = arow[0] * Kbase[i];
        for (int k = 1; k < s; ++k) acc += arow[k] * Kbase[(int64_t)k * FN + i];
        out[i] = u[i] + r->pb.dt * acc;
    }
}

/* Rsync: standard periodic right-hand side of the global field X (F x N).  */
static void rhs_sync_field(const orc_run* r, const double* X, double* out) {
    const int64_t N = r->N, E = N + 2 * r->H;
    double* g[MAXQ];
    double* vown[MAXF];
    double* K[MAXF];
    for (int k = 0; k < r->nq; ++k) g[k] = r->ext + (int64_t)k * E;
    double* lam = r->ext + (int64_t)r->nq * E;
    for (int64_t e = 0; e < E; ++e) {
        int64_t x = wrap(e - r->H, N);
        double q[MAXF], gv[MAXQ];
        for (int f = 0; f < r->F; ++f) q[f] = X[(int64_t)f * N + x];
        quantities(&r->pb, q, gv);
        for (int k = 0; k < r->nq; ++k) g[k][e] = gv[k];
        lam[e] = is_weno(&r->pb) ? wave_speed(&r->pb, q) : 0.0;
    }
    for (int f = 0; f < r->F; ++f) {
        vown[f] = (double*)X + (int64_t)f * N;
        K[f] = out + (int64_t)f * N;
    }
    rhs_region(&r->pb, 0, N, g, lam, vown, K, NULL);
}

/* Fill the synchronous stage cache G[m][1..S-1] from G[m][0] = u^m. */
static void fill_stage_cache(orc_run* r, int64_t m) {
    const int64_t FN = (int64_t)r->F * r->N;
    for (int s = 1; s < r->S; ++s) {
        rhs_sync_field(r, Gptr(r, m, s - 1), r->Rg + (int64_t)(s - 1) * FN);
        stage_combine(r, Gptr(r, m, 0), r->Rg, r->tb.a[s], s, Gptr(r, m, s));
    }
}

/* AT/AS right-hand side of stage s at PE p's own points. */
static void rhs_pe(orc_run* r, int64_t p, int s, const double* V, double* Kout) {
    const int64_t N = r->N;
    const int H = r->H, F = r->F, nq = r->nq;
    const int64_t lo = pe_lo(r, p), hi = pe_lo(r, p + 1), np = hi - lo, E = np + 2 * H;
    double* g[MAXQ];
    double* vown[MAXF];
    double* K[MAXF];
    for (int k = 0; k < nq; ++k) g[k] = r->ext + (int64_t)k * E;
    double* lam = r->ext + (int64_t)nq * E;
    for (int64_t e = 0; e < E; ++e) {
        int64_t x = wrap(lo - H + e, N);
        double q[MAXF], gv[MAXQ];
        if (e >= H && e < H + np) {                   /* own point: stage state */
            for (int f = 0; f < F; ++f) q[f] = V[(int64_t)f * N + x];
            quantities(&r->pb, q, gv);
            for (int k = 0; k < nq; ++k) g[k][e] = gv[k];
            lam[e] = is_weno(&r->pb) ? wave_speed(&r->pb, q) : 0.0;
            continue;
        }
        /* halo point: time-extrapolated synchronous stage quantities */
        int side = e < H ? 0 : 1;
        int k = r->keff[p * 2 + side];
        double w[MAXJ];
        orc_extrap_weights(r->J, k, w);
        double acc[MAXQ];
        int first = 1;
        for (int l = 0; l < r->J; ++l) {
            if (w[l] == 0.0) continue;
            const double* Gl = Gptr(r, r->n - k - l, s);
            for (int f = 0; f < F; ++f) q[f] = Gl[(int64_t)f * N + x];
            quantities(&r->pb, q, gv);
            for (int kk = 0; kk < nq; ++kk) {
                if (first) acc[kk] = w[l] * gv[kk];
                else acc[kk] += w[l] * gv[kk];
            }
            first = 0;
        }
        for (int kk = 0; kk < nq; ++kk) g[kk][e] = acc[kk];
        if (is_weno(&r->pb)) {
            /* wave speed from the freshest delayed level (no extrapolation) */
            const double* G0 = Gptr(r, r->n - k, s);
            for (int f = 0; f < F; ++f) q[f] = G0[(int64_t)f * N + x];
            lam[e] = wave_speed(&r->pb, q);
        } else {
            lam[e] = 0.0;
        }
    }
    /* own state and output slices */
    double* vbuf = (double*)malloc(sizeof(double) * (size_t)(F * np));
    double* kbuf = (double*)malloc(sizeof(double) * (size_t)(F * np));
    for (int f = 0; f < F; ++f) {
        vown[f] = vbuf + (int64_t)f * np;
        K[f] = kbuf + (int64_t)f * np;
        for (int64_t j = 0; j < np; ++j) vown[f][j] = V[(int64_t)f * N + lo + j];
    }
    rhs_region(&r->pb, lo, np, g, lam, vown, K,
               is_weno(&r->pb) ? r->flux + (lo + p) * F : NULL);
    for (int f = 0; f < F; ++f)
        for (int64_t j = 0; j < np; ++j) Kout[(int64_t)f * N + lo + j] = K[f][j];
    free(vbuf);
    free(kbuf);
}

int orc_create(const orc_problem* pb, const double* q0, orc_run** out) {
    int err = validate(pb);
    if (err) return err;
    orc_run* r = (orc_run*)calloc(1, sizeof(orc_run));
    if (!r) return ORC_ENOMEM;
    r->pb = *pb;
    get_tableau(pb->rk, &r->tb);
    r->F = orc_nfields(pb->pde);
    r->H = orc_halo_width(pb->scheme);
    r->J = orc_levels(pb->scheme, pb->mode, pb->at_levels);
    r->S = r->tb.S;
    r->D = pb->mode == ORC_SYNC ? 1 : pb->kmax + r->J;
    r->nq = nquant(pb);
    r->N = pb->n;
    const int64_t FN = (int64_t)r->F * r->N;
    r->G = (double*)calloc((size_t)(r->D * r->S) * (size_t)FN, sizeof(double));
    r->K = (double*)calloc((size_t)r->S * (size_t)FN, sizeof(double));
    r->V = (double*)calloc((size_t)FN, sizeof(double));
    r->unew = (double*)calloc((size_t)FN, sizeof(double));
    r->Rg = (double*)calloc((size_t)r->S * (size_t)FN, sizeof(double));
    r->ext = (double*)calloc((size_t)(r->nq + 1) * (size_t)(r->N + 2 * r->H), sizeof(double));
    r->flux = (double*)calloc((size_t)(r->N + pb->p) * (size_t)r->F, sizeof(double));
    r->keff = (int*)calloc((size_t)pb->p * 2, sizeof(int));
    if (!r->G || !r->K || !r->V || !r->unew || !r->Rg || !r->ext || !r->flux || !r->keff) {
        orc_free(r);
        return ORC_ENOMEM;
    }
    r->n = 0;
    memcpy(Gptr(r, 0, 0), q0, sizeof(double) * (size_t)FN);
    if (pb->mode != ORC_SYNC) fill_stage_cache(r, 0);
    *out = r;
    return ORC_OK;
}

void orc_free(orc_run* r) {
    if (!r) return;
    free(r->G); free(r->K); free(r->V); free(r->unew); free(r->Rg); free(r->ext);
    free(r->flux); free(r->keff); free(r->drawn); free(r->eff); free(r->ov);
    free(r);
}

int orc_set_history(orc_run* r, int n_levels, const double* levels, int64_t n_current) {
    if (n_levels < 1 || n_levels > r->D || n_current < n_levels - 1) return ORC_EINVAL;
    const int64_t FN = (int64_t)r->F * r->N;
    r->n = n_current;
    for (int i = 0; i < n_levels; ++i) {
        int64_t m = n_current - (n_levels - 1) + i;
        memcpy(Gptr(r, m, 0), levels + (int64_t)i * FN, sizeof(double) * (size_t)FN);
        if (r->pb.mode != ORC_SYNC) fill_stage_cache(r, m);
    }
    return ORC_OK;
}

int64_t orc_current_step(const orc_run* r) { return r->n; }

static int log_delays(orc_run* r, int64_t step, const int* drawn, const int* eff) {
    const int64_t P2 = (int64_t)r->pb.p * 2;
    if (step >= r->log_cap) {
        int64_t cap = r->log_cap ? r->log_cap : 64;
        while (cap <= step) cap *= 2;
        uint8_t* d = (uint8_t*)realloc(r->drawn, (size_t)(cap * P2));
        if (!d) return ORC_ENOMEM;
        r->drawn = d;
        uint8_t* e = (uint8_t*)realloc(r->eff, (size_t)(cap * P2));
        if (!e) return ORC_ENOMEM;
        r->eff = e;
        memset(r->drawn + r->log_cap * P2, 0xff, (size_t)((cap - r->log_cap) * P2));
        memset(r->eff + r->log_cap * P2, 0xff, (size_t)((cap - r->log_cap) * P2));
        r->log_cap = cap;
    }
    for (int64_t i = 0; i < P2; ++i) {
        r->drawn[step * P2 + i] = (uint8_t)drawn[i];
        r->eff[step * P2 + i] = (uint8_t)eff[i];
    }
    if (step + 1 > r->log_n) r->log_n = step + 1;
    return ORC_OK;
}

int orc_step(orc_run* r, int n_steps) {
    const orc_problem* pb = &r->pb;
    const int64_t N = r->N, FN = (int64_t)r->F * N, P = pb->p;
    int* drawn = (int*)malloc(sizeof(int) * (size_t)(2 * P));
    if (!drawn) return ORC_ENOMEM;
    for (int it = 0; it < n_steps; ++it) {
        const int64_t n = r->n;
        /* 1. delays (Sec. 2.1): one draw per PE (or side, or boundary) */
        for (int64_t p = 0; p < P; ++p) {
            for (int side = 0; side < 2; ++side) {
                int k;
                if (r->ov && n >= r->ov_step0 && n < r->ov_step0 + r->ov_n) {
                    k = r->ov[((n - r->ov_step0) * P + p) * 2 + side];
                } else if (pb->granularity == ORC_PER_PE) {
                    k = orc_draw(pb, n, p, 0);
                } else if (pb->granularity == ORC_PER_PE_SIDE) {
                    k = orc_draw(pb, n, p, side);
                } else {
                    k = orc_draw(pb, n, side == 0 ? p : (p + 1) % P, 0);
                }
                int ke;
                if (pb->mode == ORC_AT) {
                    ke = k;
                    if (ke > n - (r->J - 1)) ke = (int)(n - (r->J - 1));
                    if (ke < 0) ke = 0;
                } else if (pb->mode == ORC_AS) {
                    ke = k < n ? k : (int)n;
                } else {
                    ke = 0;
                }
                drawn[p * 2 + side] = k;
                r->keff[p * 2 + side] = ke;
            }
        }
        int err = log_delays(r, n, drawn, r->keff);
        if (err) { free(drawn); return err; }
        /* 2. stages (eq. rk1) */
        const double* un = Gptr(r, n, 0);
        for (int s = 0; s < r->S; ++s) {
            stage_combine(r, un, r->K, r->tb.a[s], s, r->V);
            double* Ks = r->K + (int64_t)s * FN;
            if (pb->mode == ORC_SYNC) {
                rhs_sync_field(r, r->V, Ks);
            } else {
                for (int64_t p = 0; p < P; ++p) rhs_pe(r, p, s, r->V, Ks);
            }
        }
        /* 3. update u^{n+1} = u^n + dt sum_s b_s K_s */
        stage_combine(r, un, r->K, r->tb.b, r->S, r->unew);
        memcpy(Gptr(r, n + 1, 0), r->unew, sizeof(double) * (size_t)FN);
        r->n = n + 1;
        if (pb->mode != ORC_SYNC) fill_stage_cache(r, n + 1);
    }
    free(drawn);
    return ORC_OK;
}

int orc_get_state(const orc_run* r, double* out) {
    memcpy(out, Gptr(r, r->n, 0), sizeof(double) * (size_t)r->F * (size_t)r->N);
    return ORC_OK;
}

int orc_get_stage_level(const orc_run* r, int64_t m, int s, double* out) {
    if (m > r->n || m <= r->n - r->D || m < 0 || s < 0 || s >= r->S) return ORC_ERANGE;
    if (r->pb.mode == ORC_SYNC && s > 0) return ORC_ERANGE;
    memcpy(out, Gptr(r, m, s), sizeof(double) * (size_t)r->F * (size_t)r->N);
    return ORC_OK;
}

int orc_get_delays(const orc_run* r, int64_t step0, int n_steps, uint8_t* drawn, uint8_t* eff) {
    const int64_t P2 = (int64_t)r->pb.p * 2;
    if (step0 < 0 || step0 + n_steps > r->log_n) return ORC_ERANGE;
    memcpy(drawn, r->drawn + step0 * P2, (size_t)(n_steps * P2));
    memcpy(eff, r->eff + step0 * P2, (size_t)(n_steps * P2));
    return ORC_OK;
}

int orc_set_override(orc_run* r, int64_t step0, int n_steps, const uint8_t* sched) {
    const int64_t P2 = (int64_t)r->pb.p * 2;
    if (n_steps < 0 || step0 < 0) return ORC_EINVAL;
    for (int64_t i = 0; i < n_steps * P2; ++i)
        if (sched[i] > r->pb.kmax) return ORC_ESTALE;
    free(r->ov);
    r->ov = NULL;
    r->ov_n = 0;
    if (n_steps == 0) return ORC_OK;
    r->ov = (uint8_t*)malloc((size_t)(n_steps * P2));
    if (!r->ov) return ORC_ENOMEM;
    memcpy(r->ov, sched, (size_t)(n_steps * P2));
    r->ov_step0 = step0;
    r->ov_n = n_steps;
    return ORC_OK;
}

int orc_get_fluxes(const orc_run* r, int pe, double* out) {
    if (pe < 0 || pe >= r->pb.p || !is_weno(&r->pb)) return ORC_EINVAL;
    int64_t lo = pe_lo(r, pe), hi = pe_lo(r, pe + 1);
    memcpy(out, r->flux + (lo + pe) * r->F, sizeof(double) * (size_t)((hi - lo + 1) * r->F));
    return ORC_OK;
}

int orc_rhs_sync(const orc_problem* pb, const double* q, double* out) {
    orc_run* r = NULL;
    orc_problem p2 = *pb;
    p2.mode = ORC_SYNC;
    int err = orc_create(&p2, q, &r);
    if (err) return err;
    rhs_sync_field(r, q, out);
    orc_free(r);
    return ORC_OK;
}
