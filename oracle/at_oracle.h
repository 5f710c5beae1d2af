/*
 * at_oracle.h -- plain, serial, FP64 CPU reference of the asynchrony-tolerant
 * (AT) Runge-Kutta step.  TEST INFRASTRUCTURE ONLY: only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this library; the
 * product path (libat, the HIP library) never does.
 *
 * What it computes, per the paper (Kumari et al., arXiv:2204.01133):
 *   - a periodic 1D field split into P processing elements (PEs), PE p owning
 *     points [floor(pN/P), floor((p+1)N/P))                  (Sec. 2.1, Fig. 1)
 *   - a random delay k~ in {0..kmax} per PE (or PE side, or boundary) and step,
 *     drawn from a counter-based generator (SplitMix64 finaliser, Steele, Lea &
 *     Flood 2014) and mapped to the requested probabilities (Sec. 2.1, Sec. 5,
 *     Table dels)
 *   - an explicit S-stage Runge-Kutta step in Butcher form (Sec. 2.3, eq. rk1)
 *     in which every stage at PE-boundary (halo) points is the synchronous
 *     stage value of the delayed global level, recomputed with standard
 *     schemes (Sec. 2.3, discussion after eq. rkat2)
 *   - AT spatial schemes: the standard central stencil (order 2/4/8) or
 *     WENO5-JS with local Lax-Friedrichs splitting (Sec. 3, eqs. Csplit, wender,
 *     omg, betaS, atRecon, idRec) applied with every delayed halo quantity
 *     replaced by its Lagrange extrapolation in time from levels n-k~-l,
 *     l = 0..J-1, to level n.  This reproduces Table A (J = 3) and eqs.
 *     atRecon / atReconR / atReconRm / atReconM / beta2AT* (J = 2).
 *   - WENO5 in interpolation form (Sec. 3, eqs. interpS, fullSten, omg, betaS):
 *     interface values of the split fluxes interpolated from point values by
 *     three quadratic candidates with ideal weights 1/16, 5/8, 5/16, then
 *     differenced as in eq. wender.  The AT form extrapolates the delayed halo
 *     values in time with two levels (the five-point stochastic stencil of eq.
 *     stenF, whose candidates are the standard ones applied to the
 *     extrapolated values).
 *   - AS mode: standard schemes used with the delayed level (J = 1, eq.
 *     async-fde, eq. asweno).  SYNC mode: the plain periodic scheme.
 *   - reactive NS in chain-rule form (form = 1, Sec. 4 after eq. convEq, and the
 *     memory-compute remark of Sec. 6): the derivatives of the convective products
 *     expanded by the chain rule into derivatives of the primitives rho, u, p, Y, so
 *     that the AT halo carries primitives (rho, u, p, T, Y) instead of fluxes.
 *   - non-periodic ends (bc = 1, the acoustic-wave case of Sec. 5.1 and the
 *     boundary remarks of Sec. 6): second-order central differences at the
 *     points closer to an end than the interior stencil reaches, second-order
 *     one-sided differences at the two end points, where the convective terms
 *     take the characteristic (LODI) form of the non-reflecting conditions the
 *     paper cites (Thompson 1987; Poinsot & Lele 1992) with the incoming wave
 *     amplitudes set to zero.  The ends are not PE boundaries: no delays.
 *
 * Pins (tests/test_oracle_*.py) fix every part above against closed forms, the
 * paper's printed stencils and tables, or brute force.  Parity unpinned: the
 * long-run accuracy of the one-step-chemistry flame (reactive NS over many
 * steps), whose terms are pinned one by one but whose composition has no closed
 * form; the detonation's composition is pinned by the Chapman-Jouguet speed.
 *
 * Errors: every int-returning function returns ORC_OK (0) or a negative code.
 * Ownership: the caller owns every pointer it passes; the run owns its own
 * memory and frees it in orc_free.
 */
#ifndef AT_ORACLE_H
#define AT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ESTALE = -3, ORC_ERANGE = -4 };

enum { ORC_PDE_ADV_DIFF = 0, ORC_PDE_ADR_LOGISTIC = 1, ORC_PDE_BURGERS = 2, ORC_PDE_EULER = 3,
       ORC_PDE_REACTIVE_EULER = 4, ORC_PDE_REACTIVE_NS = 5 };
enum { ORC_FD2 = 0, ORC_FD4 = 1, ORC_FD8 = 2, ORC_WENO5 = 3, ORC_WENO5I = 4 };
enum { ORC_SYNC = 0, ORC_AS = 1, ORC_AT = 2 };
enum { ORC_FE = 0, ORC_RK2 = 1, ORC_SSPRK3 = 2, ORC_RK4 = 3 };
enum { ORC_PER_PE = 0, ORC_PER_PE_SIDE = 1, ORC_PER_BOUNDARY = 2 };

typedef struct orc_problem {
    int32_t pde, scheme, mode, rk, granularity, kmax;
    int64_t n;            /* grid points N                                     */
    int32_t p;            /* number of PEs, 1 <= P <= N                         */
    int32_t n_cdf;        /* 0: uniform on {0..kmax}; else == kmax               */
    int32_t at_levels;    /* J, time levels of the AT extrapolation; 0: default  */
    int32_t bc;           /* 0: periodic; 1: two physical ends with non-reflecting
                             characteristic conditions (reactive NS, central FD)  */
    int32_t form;         /* reactive NS: 0 = the convective fluxes differentiated
                             (AT on C1..C4); 1 = chain rule on the primitives (AT on
                             rho, u, p, T, Y), Sec. 4 after eq. convEq             */
    int32_t pad_form;
    uint64_t cdf[16];     /* cumulative thresholds on a 2^32 scale               */
    double x0, lx, dt;
    double c, alpha, r, gamma, q, ea, b, mu, pr, le, weno_eps;
    uint64_t seed;
    int64_t problem_id;
} orc_problem;

typedef struct orc_run orc_run;

int  orc_create(const orc_problem* pb, const double* q0 /* F x N, SoA */, orc_run** out);
void orc_free(orc_run* r);
/* Replace the history: n_levels levels (oldest first, each F x N) ending at
 * step n_current; the synchronous stage cache of each level is recomputed. */
int  orc_set_history(orc_run* r, int n_levels, const double* levels, int64_t n_current);
int  orc_step(orc_run* r, int n_steps);
int64_t orc_current_step(const orc_run* r);
int  orc_get_state(const orc_run* r, double* out /* F x N */);
/* Synchronous stage s (0-based) of level m, if still held. */
int  orc_get_stage_level(const orc_run* r, int64_t m, int s, double* out);
int  orc_get_delays(const orc_run* r, int64_t step0, int n_steps, uint8_t* drawn, uint8_t* eff);
int  orc_set_override(orc_run* r, int64_t step0, int n_steps, const uint8_t* sched /* n x P x 2 */);
/* Interface fluxes of PE pe from the last AT/AS right-hand side (WENO only):
 * (n_pe + 1) x F values, interface i between own points i-1 and i. */
int  orc_get_fluxes(const orc_run* r, int pe, double* out);

/* pieces exposed for pinning */
uint64_t orc_mix64(uint64_t z);
int  orc_draw(const orc_problem* pb, int64_t step, int64_t idx, int side);
int  orc_extrap_weights(int J, int k, double* w);
int  orc_rhs_sync(const orc_problem* pb, const double* q, double* out);
/* Convective time derivatives of (rho, rho u, rho E, rho Y) at an end point in the
 * characteristic (LODI) form, from the primitives (rho, u, p, Y) and their x
 * derivatives; side 0 left, 1 right; drop = 1 sets the incoming amplitudes to 0. */
int  orc_lodi(const orc_problem* pb, int side, int drop, const double* prim, const double* dprim,
              double* out);
int  orc_nfields(int pde);
/* WENO5 interpolation (eqs. interpS, omg, betaS) of the value at the right edge of v[2]
 * from v[0..4]; beta (may be null) receives the three smoothness indicators. */
double orc_weno_interp(double eps, const double* v, double* beta);
int  orc_halo_width(int scheme);
int  orc_levels(int scheme, int mode, int at_levels);

#ifdef __cplusplus
}
#endif
#endif
