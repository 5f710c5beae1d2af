/*
 * at.h -- C ABI of libat, the MI355X (gfx950) implementation of the
 * asynchrony-tolerant (AT) multi-stage Runge-Kutta step of Kumari et al.,
 * "Evaluation of finite difference based asynchronous partial differential
 * equations solver for reacting flows" (arXiv:2204.01133).
 *
 * The operation (Sec. 2.1-2.3 and Sec. 3 of the paper): a periodic 1D problem
 * of N points is split into P processing elements (PEs).  Every step draws a
 * delay k~ in {0..kmax} per PE (Sec. 2.1; probabilities of Table dels) and
 * advances all S stages of an explicit RK scheme (eq. rk1).  At PE-boundary
 * halo points each stage uses the synchronous stage values of the delayed
 * levels n-k~-l, l = 0..J-1, extrapolated in time to level n (Table A for the
 * central schemes, eqs. atRecon/beta2AT* for AT-WENO), the multi-stage
 * procedure of Sec. 2.3.  Interior points use the standard central
 * difference (order 2, 4 or 8) or WENO5-JS with local Lax-Friedrichs flux
 * splitting (eqs. Csplit, wender, omg, betaS, idRec).
 *
 * Memory and streams: the caller owns every device buffer and the HIP stream.
 * at_init computes the size of ONE device workspace; the caller allocates it
 * (e.g. with torch) and hands it over with at_bind.  The library never
 * allocates or frees device memory.  Calls that take the context are
 * stream-ordered and asynchronous unless stated; one context per stream, no
 * internal locking.  Host pointers may be pageable.
 *
 * Errors: every int-returning entry point returns AT_OK (0) or a negative
 * AT_E* code; no exception crosses the ABI.  at_strerror gives a static
 * string, at_last_error the context's last detailed message.
 */
#ifndef AT_H
#define AT_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum at_status {
    AT_OK = 0,
    AT_EINVAL = -1,        /* bad descriptor, size or argument                          */
    AT_EUNSUPPORTED = -2,  /* valid combination the library does not run (e.g. PE too big) */
    AT_ESTATE = -3,        /* call order (not bound, state not set, mid-step)           */
    AT_EHIP = -4,          /* HIP runtime error; text in at_last_error                  */
    AT_ESTALE = -5,        /* delay override asks for data older than the ring holds    */
    AT_ERANGE = -6         /* step or problem index outside what is held                */
};

enum at_pde { AT_PDE_ADV_DIFF = 0, AT_PDE_ADR_LOGISTIC = 1, AT_PDE_BURGERS = 2, AT_PDE_EULER = 3,
              AT_PDE_REACTIVE_EULER = 4, AT_PDE_REACTIVE_NS = 5 };
enum at_scheme { AT_FD2 = 0, AT_FD4 = 1, AT_FD8 = 2, AT_WENO5 = 3, AT_WENO5I = 4 };
enum at_mode { AT_SYNC = 0, AT_AS = 1, AT_AT = 2 };
enum at_rk { AT_FE = 0, AT_RK2 = 1, AT_SSPRK3 = 2, AT_RK4 = 3 };
enum at_granularity { AT_PER_PE = 0, AT_PER_PE_SIDE = 1, AT_PER_BOUNDARY = 2 };
enum at_precision { AT_FP64 = 0, AT_FP32C = 1, AT_FP32 = 2 };

/*
 * One periodic problem (plain old data).
 *   pde/scheme   PDE and spatial scheme; central FD with advection-diffusion(-
 *                logistic) and one-step-chemistry Navier-Stokes, WENO5 with
 *                linear advection (alpha = 0), Burgers, Euler, reactive Euler.
 *                AT_WENO5 reconstructs the interface fluxes (Jiang-Shu candidates,
 *                ideal weights 1/10, 3/5, 3/10); AT_WENO5I interpolates them from the
 *                point values (Sec. 3, eqs. interpS, fullSten: ideal weights 1/16,
 *                5/8, 5/16; a second-order flux derivative).
 *   mode         AT (extrapolated delayed halos), AS (standard scheme on the
 *                delayed level, eq. async-fde / asweno), SYNC (delay 0).
 *   rk           Butcher tableau: forward Euler, RK2 (eq. rk2), SSP-RK3, RK4.
 *   granularity  one delay per PE (both sides), per PE side, or per boundary.
 *   precision    FP64; FP32C = FP32 arithmetic with the state kept as a
 *                compensated hi+lo pair (TwoSum update) and FP64 temperature
 *                inversion and Arrhenius rate; FP32 = the same without
 *                persisting lo between steps.
 *   kmax         largest delay (0..15).  n_cdf = 0: uniform on {0..kmax};
 *                n_cdf = kmax: delay k is the number of thresholds cdf[i]
 *                (i < kmax, 2^32 scale) at or below the draw's top 32 bits.
 *   at_levels    J, time levels of the AT extrapolation (0: 3 for FD4/FD8,
 *                2 for FD2 and the WENO schemes; 2 levels make the AT-WENO
 *                interpolation form the five-point stencil of eq. stenF).
 *   n, p         points and PEs, 1 <= p <= n; PE k owns [floor(kn/p), floor((k+1)n/p)).
 *   form         reactive NS: 0 = the convective fluxes are differentiated (the AT
 *                halo carries C1..C4, u, T, Y); 1 = the chain rule expands their
 *                derivatives into those of the primitives (Sec. 4 after eq. convEq:
 *                the AT halo carries rho, u, p, T, Y); periodic problems only.
 *   x0, lx, dt   grid x_j = x0 + (j + 1/2) lx/n; constant time step.
 *   c, alpha, r  advection speed, diffusivity, logistic rate.
 *   gamma, q, ea, b, mu, pr, le  gas constant ratio (R = 1), heat release,
 *                activation energy, pre-exponential factor, viscosity, Prandtl
 *                and Lewis numbers (one-step chemistry, E = T/(gamma-1) +
 *                u^2/2 + q Y, rate -b rho Y exp(-ea/T)).
 *   weno_eps     epsilon of the WENO weights (eq. omg), e.g. 1e-6.
 *   seed, problem_id  key of the counter-based delay generator (SplitMix64
 *                finaliser; draw for (step, pe, side) as in the oracle docs).
 *   bc           0: periodic.  1: two physical ends with non-reflecting
 *                characteristic conditions (the acoustic-wave case of Sec. 5.1;
 *                boundary remarks of Sec. 6): second-order one-sided differences
 *                and the characteristic (LODI) form of the convective terms with
 *                the incoming waves removed at the two end points, second-order
 *                central differences at the other points the interior stencil
 *                cannot reach.  Reactive NS with central FD only; the first and the
 *                last PE must hold max(4, S*H) points (AT_EUNSUPPORTED otherwise).
 */
typedef struct at_problem_desc {
    int32_t pde, scheme, mode, rk, granularity, precision;
    int32_t kmax, at_levels, n_cdf, bc;
    int64_t n;
    int32_t p, form;
    uint64_t cdf[16];
    double x0, lx, dt;
    double c, alpha, r, gamma, q, ea, b, mu, pr, le, weno_eps;
    uint64_t seed;
    int64_t problem_id;
} at_problem_desc;

/*
 * Launch options (all 0 = defaults chosen by the planner).
 *   tile_points     largest number of points of one tile (work item); PEs are
 *                   packed whole into tiles, a PE may not exceed it.  By default
 *                   the small-tile capacity, with PEs packed only up to about two
 *                   tiles per compute unit for workloads too small to fill the GPU.
 *   persistent      batched form: 1 = persistent grid (grid-stride over the
 *                   work list), 0 = one workgroup per tile, -1 = planner's choice
 *                   (one workgroup per tile, which measured faster everywhere).
 *   grid_per_cu     persistent grid size = grid_per_cu x 256 compute units
 *                   (0 = 6, the workgroups per CU of the default LDS budget).
 *   graph_steps     batched form: steps per captured HIP graph (0 = plain launches).
 *   xcd_remap       1 = XCD-aware tile order (consecutive tiles on one XCD).
 *   log_steps       capacity, in steps, of the device delay log (0 = off).
 *   override_steps  capacity, in steps, of the delay-override buffer (0 = off).
 *   stage_api       1 = reserve the stage buffers that at_rk_stage needs.
 *   lds_budget      bytes of LDS per tile the planner packs PEs up to (0 = the
 *                   default of the kernel: 26 KiB, 6 workgroups per compute unit,
 *                   for the FP32 scalar finite-difference kernels of order 2 and 4,
 *                   whose whole-step kernel is held to the registers of 6 waves per
 *                   SIMD; 40 KiB, 4 workgroups, otherwise); a tile of one PE may
 *                   exceed it (up to the 160 KiB of a compute unit).
 *   tile_class      0 = tiles of the small points-per-thread class of the kernel (the
 *                   default), 1 = every tile of the large class (twice the points per
 *                   thread, twice the points per tile).
 *   halo_lds        scalar finite-difference kinds: 0 = the delayed halo strips are
 *                   loaded into registers and extrapolated in time once per step by
 *                   one lane per PE side (the default); 1 = they are copied into LDS
 *                   by every lane and extrapolated where each stage reads them.  The
 *                   other kinds always copy them into LDS.  The results are the same
 *                   bit for bit.
 */
typedef struct at_run_opts {
    int32_t tile_points, persistent, grid_per_cu, graph_steps;
    int32_t xcd_remap, log_steps, override_steps, stage_api;
    int32_t lds_budget;
    int32_t tile_class, halo_lds;
    int32_t reserved[5];
} at_run_opts;

typedef struct at_ctx at_ctx;

/* (Sec. 2.1, Fig. 1: the PE decomposition with buffer points; Sec. 2.2: the
 * delayed time levels the AT halo needs.)  Validate the problems, plan the PE
 * partitions, the tiles, the ring of delayed levels and the work list; no device memory is
 * touched.  *workspace_bytes receives the size of the device workspace.
 * Errors: AT_EINVAL (descriptor), AT_EUNSUPPORTED (e.g. a PE larger than a tile). */
int at_init(const at_problem_desc* probs, int n_probs, const at_run_opts* opts, at_ctx** out,
            size_t* workspace_bytes);

/* (Sec. 2.1-2.2: the states and the ring of past boundary levels live here.)
 * Hand over the caller-owned device workspace (>= workspace_bytes, 256-byte
 * aligned) and the HIP stream (hipStream_t, NULL = default stream) on the
 * current device.  Uploads the problem tables (stream-ordered) and creates the
 * side streams and events of at_batch_step (one per kernel variant after the
 * first).  Binding forgets all progress (as at_reset).  Errors: AT_EINVAL, AT_EHIP. */
int at_bind(at_ctx* ctx, void* d_workspace, size_t bytes, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): like at_bind, but the
 * workspace is the library's own device scratch, a static array of
 * AT_SCRATCH_BYTES (128 MiB) per device, held by each device the library runs on
 * until the process ends.  Calls no hipMalloc, hipFree or other allocating routine,
 * creates no stream, event or graph: the kernel groups of a batched step run one
 * after another on the given stream and at_batch_step launches them directly
 * (graph_steps is ignored).  The caller still passes inputs and outputs
 * (at_set_state, at_get_state).  One context holds a device's scratch at a time:
 * binding another context to it on the same device makes the earlier one fail
 * with AT_ESTATE; calls of contexts that overlap in time on one device race.
 * The scratch keeps the last context's contents; nothing in it needs clearing
 * (every word a kernel reads was written earlier in the same binding).  Like
 * at_bind, binding forgets all progress (as at_reset).
 * Errors: AT_EUNSUPPORTED (workspace_bytes above AT_SCRATCH_BYTES, or a device
 * index above 63), AT_EHIP. */
#define AT_SCRATCH_BYTES ((size_t)128 << 20)
int at_bind_scratch(at_ctx* ctx, void* hip_stream);

/* (Sec. 2.3, eq. rk1: u^0, the state the first step starts from.)
 * Set problem `prob`'s level-0 state: F x N doubles (structure of arrays,
 * field-major) on the host (q_on_device = 0; copied before return) or on the
 * device (stream-ordered).  Resets the step counter of the context to 0 when
 * called before the first step; AT_ESTATE after stepping (use at_reset). */
int at_set_state(at_ctx* ctx, int prob, const double* q, int q_on_device);

/* (Sec. 2.1: the delays are bounded by the levels held, so a new start holds none.)
 * Forget all progress: step counter and stage pointer to 0; states must be set again. */
int at_reset(at_ctx* ctx);

/* (Sec. 2.3, eqs. rk1, rkat1: one stage, K_s from the AT halo of the delayed
 * levels' synchronous stage values.)
 * One RK stage (1-based, 1..S) of the current step for every problem: draws
 * the delays and builds the level's halo strips at stage 1, keeps stage
 * right-hand sides in the workspace, and at stage S forms u^{n+1} and
 * advances the step.  Stages must be called in order.  Needs stage_api.
 * Results equal at_step's.  Errors: AT_ESTATE, AT_EINVAL, AT_EHIP. */
int at_rk_stage(at_ctx* ctx, int stage);

/* (Sec. 2.3, eq. rk1: all S stages and the update, with the AT schemes of Sec. 2.2
 * and Sec. 3 at PE boundaries.)
 * Plain form: n_steps steps, each one fused all-stage kernel launch per problem. */
int at_step(at_ctx* ctx, int n_steps);

/* (Sec. 2.3, eq. rk1, as at_step.)
 * Batched form: n_steps steps, each one launch per kernel variant over the
 * work list of all problems (persistent or one workgroup per tile), replayed
 * from captured HIP graphs of graph_steps steps when enabled.  The launches of
 * one step run concurrently: the first on the context's stream, the others on
 * library-owned streams (created by at_bind, destroyed by at_free) that fork
 * from it and join back into it with events, so the call stays ordered on the
 * context's stream.  Errors: AT_ESTATE, AT_EINVAL, AT_EHIP. */
int at_batch_step(at_ctx* ctx, int n_steps);

/* (Sec. 2.3, eq. rk1: u^n.)
 * Copy problem `prob`'s current state out as F x N doubles (hi + lo for the
 * FP32 forms).  out_on_device = 0: host buffer, synchronises the stream. */
int at_get_state(at_ctx* ctx, int prob, double* out, int out_on_device);

/* (Sec. 2.1 and Table dels: the delay k~ of each PE and step.)
 * Delays drawn and used (effective, clamped to the held history) for steps
 * [step0, step0 + n_steps), each P x 2 (PE, side) bytes; needs log_steps and
 * the steps to be inside the logged window.  Synchronises the stream. */
int at_get_delays(at_ctx* ctx, int prob, int64_t step0, int n_steps, uint8_t* drawn,
                  uint8_t* effective);

/* (Sec. 2.1: the delays k~, here prescribed instead of drawn.)
 * Replace the drawn delays of problem `prob` for steps [step0, step0+n_steps)
 * by sched (n_steps x P x 2 bytes, host).  Values above kmax: AT_ESTALE (the
 * ring holds only kmax + J levels).  n_steps = 0 clears.  Needs override_steps. */
int at_set_delay_override(at_ctx* ctx, int prob, const uint8_t* sched, int64_t step0,
                          int n_steps);

/* (No passage: interface housekeeping.)  Wait for the context's stream. */
int at_sync(at_ctx* ctx);

/* (Sec. 2.1: sizes of the partition and its work.)
 * Introspection: AT_Q_* keys below; value out.  Errors: AT_EINVAL. */
enum at_query_key {
    AT_Q_STEP = 0,            /* current step n                                     */
    AT_Q_NUM_TILES = 1,       /* work items over all problems                        */
    AT_Q_NUM_GROUPS = 2,      /* kernel variants (launches per batched step)         */
    AT_Q_TOTAL_POINTS = 3,    /* sum of N                                            */
    AT_Q_STATE_BYTES = 4,     /* algorithmic state bytes moved per step (read+write) */
    AT_Q_STAGES = 5,          /* RK stages of problem 0                              */
    AT_Q_LDS_BYTES = 6,       /* largest dynamic LDS of a launch                     */
    AT_Q_STRIP_BYTES = 7,     /* ring strip bytes written per step                   */
    AT_Q_NUM_PES = 8          /* sum of P                                            */
};
int at_query(const at_ctx* ctx, int key, int64_t* value);

/* (No passage: interface housekeeping.)  Device stream the last launches went to
 * (for event timing on that stream). */
void* at_stream(const at_ctx* ctx);

/* (No passage: interface housekeeping.)  Text of an error code; of the context's
 * last error (its planner or HIP message; with a null context, the planner's
 * message of the calling thread's last failed at_init, which returns no context);
 * release of the context and of what at_bind created (streams, events, graphs;
 * the caller's workspace stays the caller's). */
const char* at_strerror(int code);
const char* at_last_error(const at_ctx* ctx);
void at_free(at_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* AT_H */
