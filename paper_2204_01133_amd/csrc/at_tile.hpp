// at_tile.hpp -- the work of one tile (a run of whole PEs of one problem) for
// one asynchrony-tolerant RK step, written once for the gfx950 kernels and for
// the bounds-checked CPU emulation used by the tests.
//
// Method (Kumari et al., arXiv:2204.01133):
//   * delays: one draw per PE / PE side / boundary and step from a counter-based
//     hash (SplitMix64 finaliser), uniform or by cumulative thresholds
//     (Sec. 2.1; Sec. 5, Table dels);
//   * multi-stage AT procedure (Sec. 2.3): the halo value of stage s at a
//     delayed level m is the synchronous stage s of the global level m; it is
//     computed once, when level m is current, from a window of 2*S*H raw
//     points around each PE boundary, and kept in a ring of per-PE "strips"
//     (S stages x H points x F fields per side) in HBM;
//   * AT halo: Lagrange extrapolation in time of the differentiated quantity
//     from levels n-k, ..., n-k-J+1 to level n with exact integer weights
//     (Table A for J = 3; eqs. atRecon, beta2AT* for J = 2);
//   * interior: central differences of order 2H (Table A's 4th order, 2nd
//     order of eq. at1, 8th order) or WENO5-JS with local Lax-Friedrichs
//     splitting (eqs. Csplit, wender, omg, betaS, idRec);
//   * RK stages in Butcher form (eq. rk1), all stages of a step fused.
//
// Data layout in LDS ("ext" positions): per PE of the tile H halo slots, its own
// points, H halo slots (concatenated); then one window of 2*S*H positions per
// PE boundary.  Own-point state and stage right-hand sides stay in registers.
#pragma once
#include <math.h>
#include <stdint.h>

#include <type_traits>

#ifdef __HIPCC__
#define AT_HD __host__ __device__
#define AT_FI __forceinline__
#else
#define AT_HD
#define AT_FI inline
#endif

// Memory that no kernel writes while it runs (problem descriptors, the tile list): on
// the GPU it is read through the constant address space, so that uniform reads of it
// are scalar loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define AT_CONST __attribute__((address_space(4)))
#else
#define AT_CONST
#endif

#ifdef AT_EMU
void at_emu_fail(const char* what, const char* file, int line, long long i, long long n);
#define AT_CHECK(c, what, i, n) \
    do { if (!(c)) at_emu_fail(what, __FILE__, __LINE__, (long long)(i), (long long)(n)); } while (0)
#else
#define AT_CHECK(c, what, i, n) ((void)0)
#endif

namespace atk {

enum Kind { K_ADR = 0, K_RNS = 1, K_WSCAL = 2, K_EUL = 3, K_REUL = 4 };
enum Pde { PDE_ADV_DIFF = 0, PDE_ADR_LOGISTIC = 1, PDE_BURGERS = 2, PDE_EULER = 3,
           PDE_REACTIVE_EULER = 4, PDE_REACTIVE_NS = 5 };
enum Mode { M_SYNC = 0, M_AS = 1, M_AT = 2 };
enum Gran { G_PE = 0, G_PE_SIDE = 1, G_BOUNDARY = 2 };

constexpr int MAXF = 4;
constexpr int MAXS = 4;
constexpr int MAXJ = 8;

// Bounds-checked in the CPU emulation, a plain pointer on the GPU.
template <class T>
struct View {
    T* p;
    int64_t n;
    AT_HD AT_FI T& operator[](int64_t i) const {
        AT_CHECK(i >= 0 && i < n, "view", i, n);
        return p[i];
    }
};

// Global-memory element access.  On the GPU the pointer is taken in the global
// address space, so the compiler emits global (not flat) loads and stores: flat
// operations also count against the LDS wait counter that every barrier drains.
// Indices are 32-bit unsigned (the planner keeps every array under 4 GiB), so with a
// uniform base the address is the scalar base plus a 32-bit vector offset (one VGPR,
// not a 64-bit address pair per access).
#if defined(__HIP_DEVICE_COMPILE__)
// byte offset of element i in 32 bits (every array is under 4 GiB), added to the base as
// an unsigned 32-bit value: the scalar-base + 32-bit vector-offset form of the access
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gptr(const T* p, uint32_t i) {
    return (const __attribute__((address_space(1))) T*)((const __attribute__((address_space(1))) char*)p +
                                                        (uint32_t)(i * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ T gld(const T* p, uint32_t i) {
    return *gptr(p, i);
}
template <class T>
__device__ __forceinline__ void gst(T* p, uint32_t i, T v) {
    *(__attribute__((address_space(1))) T*)gptr((const T*)p, i) = v;
}
#else
template <class T>
inline T gld(const T* p, uint32_t i) { return p[i]; }
template <class T>
inline void gst(T* p, uint32_t i, T v) { p[i] = v; }
#endif

// Direct global-to-LDS copy of one 32-bit word per lane: lane j of a wave writes word
// j of the wave's LDS block, whose base must be the same across the wave (the LDS
// address register of the instruction is per wave).  The copy holds no register and
// completes on the vector-memory counter, so the barrier after it must drain that
// counter too.  On the host the lane writes its word directly.
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ void lds_copy_word(float* lds_wave, int lane, const float* g, uint32_t i) {
    (void)lane;
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)gptr(g, i),
                                     (__attribute__((address_space(3))) void*)lds_wave, 4, 0, 0);
}
#else
inline void lds_copy_word(float* lds_wave, int lane, const float* g, uint32_t i) { lds_wave[lane] = g[i]; }
#endif

// A scheduling fence: the compiler moves no instruction across it (keeps the loads of a
// group of points from being hoisted above the arithmetic of the previous group, which
// would need more registers than the occupancy target allows).  Nothing on the host.
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }
#else
inline void sched_fence() {}
#endif

// Wait for the wave's vector-memory loads (vmcnt(0) on the GPU; nothing on the host).
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ void vm_drain() { __builtin_amdgcn_s_waitcnt(0x0F70); }
#else
inline void vm_drain() {}
#endif

// Bounds-checked (emulation) view of a global array.
template <class T>
struct GView {
    T* p;
    int64_t n;
    AT_HD AT_FI T ld(int64_t i) const {
        AT_CHECK(i >= 0 && i < n, "global view", i, n);
        return gld(p, (uint32_t)i);
    }
    AT_HD AT_FI void st(int64_t i, T v) const {
        AT_CHECK(i >= 0 && i < n, "global view", i, n);
        gst(p, (uint32_t)i, v);
    }
};

// Device-resident description of one problem (built by the planner).
struct ProbDev {
    int64_t n;
    int32_t p, pde, mode, gran, kmax, J, D, n_cdf, keep_lo, S, F;
    int32_t bc;              // 1: non-periodic ends with non-reflecting conditions
    int32_t interp;          // WENO kinds: 1 = interpolation form (AT_WENO5I)
    int32_t form, pad_form;  // reactive NS: 1 = chain rule on the primitives
    uint64_t cdf[16];
    uint64_t seed;
    int64_t pid;
    double dt, inv_dx, inv_dx2;
    double c, alpha, r, gamma, q, ea, b, mu, kappa, rhoD, eps;
    double a[MAXS][MAXS];
    double bw[MAXS];
    double lin_p[4], lin_m[4];   // scalar FD kind: weights of u_{i+o} - u_i and u_{i-o} - u_i
    // FP32 copies of the constants of the FP32 forms, rounded on the host (so that they
    // arrive in scalar registers): lin_p, lin_m, their sum, the logistic rate (0 unless the
    // PDE has the logistic term), dt, c, r, alpha, 1/dx, 1/dx^2
    float lpf[4], lmf[4];
    float c0f, rlf, dtf, cf, rf, alphaf, inv_dxf, inv_dx2f;
    // memory (device addresses; host addresses in the emulation)
    void* st_hi[2];          // state ping-pong: F x N (FP64 value or FP32 hi)
    void* st_lo[2];          // FP32 forms: lo parts
    void* ring;              // strip ring: D x P x 2 records of rec_bytes
    const int32_t* peoff;    // first point of PE p, p = 0..P (floor(p N / P))
    double inv_p;            // 1 / P
    int64_t rec_bytes;
    void* kbuf;              // stage right-hand sides for the per-stage entry point
    uint8_t* ov;             // delay override [ov_n][P][2]
    int64_t ov_step0, ov_n;
    uint8_t* log_drawn;      // delay log ring [log_cap][P][2]
    uint8_t* log_eff;
    int64_t log_cap;
    int64_t kbuf_len;        // elements (emulation bounds)
};

struct Tile {
    int32_t prob, pe0, npe, npts;
    int64_t lo;              // first global point of the tile
};

enum KFlags { KF_STAGE_IO = 1, KF_LOG = 2, KF_XCD = 4, KF_HALO_LDS = 8 };

// Physics parameters of one problem, hoisted into registers at the start of a
// tile (uniform across the workgroup: scalar registers on the GPU).
struct PhysP {
    int pde;
    int interp;           // WENO kinds: interpolation form of the interface values
    int form;             // reactive NS: chain rule on the primitives
    double c, alpha, r, gamma, q, ea, b, mu, kappa, rhoD, eps, inv_dx, inv_dx2, dt;
    float cf, alphaf, rf, inv_dxf, inv_dx2f;     // FP32 copies for the FP32 forms
    double lp[4], lm[4];                           // scalar FD kind: combined stencil
    float lpf[4], lmf[4];
    float c0f;                                     // FP32 scalar kind: sum of lpf and lmf
    float rlf;                                     // FP32 scalar kind: logistic rate (0 without)
    float dtf;                                     // FP32 forms: dt
    // WENO kinds: eps of the weights in the scaled form of weno5_corr (48/13 eps) and
    // dx^-1 / 2 (the interface flux is kept without its factor 1/2), FP64 and FP32
    double epsw, hidx;
    float epswf, hidxf;
};

#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
    union { double d; int i[2]; } u;
    u.d = v;
    u.i[0] = __builtin_amdgcn_readfirstlane(u.i[0]);
    u.i[1] = __builtin_amdgcn_readfirstlane(u.i[1]);
    return u.d;
}
__device__ __forceinline__ float uni(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ int64_t uni(int64_t v) {
    union { int64_t l; int i[2]; } u;
    u.l = v;
    u.i[0] = __builtin_amdgcn_readfirstlane(u.i[0]);
    u.i[1] = __builtin_amdgcn_readfirstlane(u.i[1]);
    return u.l;
}
#else
inline int uni(int v) { return v; }
inline float uni(float v) { return v; }
inline double uni(double v) { return v; }
inline int64_t uni(int64_t v) { return v; }
#endif

template <class T>
AT_HD AT_FI T* uni_ptr(T* p) { return (T*)(uintptr_t)uni((int64_t)(uintptr_t)p); }

// A register copy of a problem descriptor whose every field is known to be the same
// across the workgroup (scalar registers on the GPU): read once at the start of a
// tile, so no later access goes back to memory.  Its arrays are only ever indexed with
// compile-time indices (a run-time index would put the copy in scratch memory), so the
// delay thresholds cdf, which the delay draw indexes at run time, are not copied.
AT_HD AT_FI ProbDev uniform_copy(const AT_CONST ProbDev& P) {
    ProbDev u;
    u.n = uni(P.n);
    u.p = uni(P.p); u.pde = uni(P.pde); u.mode = uni(P.mode); u.gran = uni(P.gran);
    u.kmax = uni(P.kmax); u.J = uni(P.J); u.D = uni(P.D); u.n_cdf = uni(P.n_cdf);
    u.keep_lo = uni(P.keep_lo); u.S = uni(P.S); u.F = uni(P.F);
    u.bc = uni(P.bc);
    u.interp = uni(P.interp);
    u.form = uni(P.form);
    u.seed = (uint64_t)uni((int64_t)P.seed);
    u.pid = uni(P.pid);
    u.dt = uni(P.dt); u.inv_dx = uni(P.inv_dx); u.inv_dx2 = uni(P.inv_dx2);
    u.c = uni(P.c); u.alpha = uni(P.alpha); u.r = uni(P.r); u.gamma = uni(P.gamma);
    u.q = uni(P.q); u.ea = uni(P.ea); u.b = uni(P.b); u.mu = uni(P.mu);
    u.kappa = uni(P.kappa); u.rhoD = uni(P.rhoD); u.eps = uni(P.eps);
    for (int i = 0; i < MAXS; ++i) {
        for (int j = 0; j < MAXS; ++j) u.a[i][j] = uni(P.a[i][j]);
        u.bw[i] = uni(P.bw[i]);
    }
    for (int i = 0; i < 4; ++i) {
        u.lin_p[i] = uni(P.lin_p[i]);
        u.lin_m[i] = uni(P.lin_m[i]);
        u.lpf[i] = uni(P.lpf[i]);
        u.lmf[i] = uni(P.lmf[i]);
    }
    u.c0f = uni(P.c0f); u.rlf = uni(P.rlf); u.dtf = uni(P.dtf); u.cf = uni(P.cf); u.rf = uni(P.rf);
    u.alphaf = uni(P.alphaf); u.inv_dxf = uni(P.inv_dxf); u.inv_dx2f = uni(P.inv_dx2f);
    for (int w = 0; w < 2; ++w) {
        u.st_hi[w] = uni_ptr(P.st_hi[w]);
        u.st_lo[w] = uni_ptr(P.st_lo[w]);
    }
    u.ring = uni_ptr(P.ring);
    u.peoff = uni_ptr(P.peoff);
    u.inv_p = uni(P.inv_p);
    u.rec_bytes = uni(P.rec_bytes);
    u.kbuf = uni_ptr(P.kbuf);
    u.ov = uni_ptr(P.ov);
    u.ov_step0 = uni(P.ov_step0); u.ov_n = uni(P.ov_n);
    u.log_drawn = uni_ptr(P.log_drawn); u.log_eff = uni_ptr(P.log_eff);
    u.log_cap = uni(P.log_cap);
    u.kbuf_len = uni(P.kbuf_len);
    return u;
}

// Butcher tableaus (eq. rk1) fixed by the stage count of the supported schemes:
// S = 1 forward Euler, 2 Heun (eq. rk2), 3 SSP-RK3, 4 classical RK4.
template <int S> struct RKTab;
template <> struct RKTab<1> {
    AT_HD static constexpr double a(int, int) { return 0.0; }
    AT_HD static constexpr double b(int) { return 1.0; }
};
template <> struct RKTab<2> {
    AT_HD static constexpr double a(int s, int i) { return (s == 1 && i == 0) ? 1.0 : 0.0; }
    AT_HD static constexpr double b(int) { return 0.5; }
};
template <> struct RKTab<3> {
    AT_HD static constexpr double a(int s, int i) { return s == 1 ? (i == 0 ? 1.0 : 0.0) : (s == 2 && i < 2 ? 0.25 : 0.0); }
    AT_HD static constexpr double b(int s) { return s == 2 ? 2.0 / 3.0 : 1.0 / 6.0; }
};
template <> struct RKTab<4> {
    AT_HD static constexpr double a(int s, int i) { return (s >= 1 && i == s - 1) ? (s == 3 ? 1.0 : 0.5) : 0.0; }
    AT_HD static constexpr double b(int s) { return (s == 1 || s == 2) ? 1.0 / 3.0 : 1.0 / 6.0; }
};

// Whether a window stage update needs a right-hand side older than the current
// stage (a_{s+1,i} != 0 for some i < s); if not, the window stage RHS are not kept.
template <int S>
AT_HD constexpr bool rk_keeps_stage_rhs() {
    for (int s = 1; s + 1 <= S - 1; ++s)
        for (int i = 0; i < s; ++i)
            if (RKTab<S>::a(s + 1, i) != 0.0) return true;
    return false;
}

struct KArgs {
    const Tile* tiles;
    const ProbDev* probs;
    const ProbDev* tprobs;    // descriptor of the problem of tiles[i] at tprobs[i]
    const int64_t* step_ptr;  // device step counter (graph replays), may be null
    int64_t step_off;
    int32_t ntiles, npts_max, npe_max, jmax;
    int32_t s_begin, s_end, flags, lds_bytes;
};

// ---------------------------------------------------------------------------
// kind traits and configuration
// ---------------------------------------------------------------------------
template <int KIND> struct KindInfo;
template <> struct KindInfo<K_ADR>   { static constexpr int F = 1, NQ = 1; static constexpr bool WENO = false, T64 = false; };
template <> struct KindInfo<K_RNS>   { static constexpr int F = 4, NQ = 7; static constexpr bool WENO = false, T64 = true; };
template <> struct KindInfo<K_WSCAL> { static constexpr int F = 1, NQ = 2; static constexpr bool WENO = true, T64 = false; };
template <> struct KindInfo<K_EUL>   { static constexpr int F = 3, NQ = 6; static constexpr bool WENO = true, T64 = false; };
template <> struct KindInfo<K_REUL>  { static constexpr int F = 4, NQ = 8; static constexpr bool WENO = true, T64 = true; };

template <int KIND_, int H_, int S_, bool F32_, int PPT_>
struct Cfg {
    static constexpr int KIND = KIND_, H = H_, S = S_, PPT = PPT_;
    static constexpr bool F32 = F32_;
    using KI = KindInfo<KIND_>;
    static constexpr int F = KI::F, NQ = KI::NQ;
    static constexpr bool WENO = KI::WENO;
    static constexpr bool HILO = F32_ && KIND_ == K_ADR;        // hi/lo difference stencils
    using lreal = typename std::conditional<F32_, float, double>::type;   // LDS values, K
    using qreal = typename std::conditional<F32_ && !KI::T64, float, double>::type;  // quantities
    static constexpr int WL = 2 * S_ * H_;                      // boundary window length
    // occupancy target of the kernel (waves per SIMD; 1 = the compiler's choice): the
    // small-tile scalar FD kernels (8 points per thread in FP32, 6 in FP64) are held to
    // 128 VGPRs (4 waves) instead of ~160 (3)
    static constexpr int WAVES_PER_EU = (KIND_ == K_ADR && PPT_ == (F32_ ? 8 : 6)) ? 4 : 1;
    // the whole-step FP32 scalar FD kernel of halo width up to 2 is held to 80 VGPRs
    // (6 waves), which its default LDS per tile (26 KiB, 6 workgroups per compute unit)
    // matches
    static constexpr int WAVES_STEP = (KIND_ == K_ADR && F32_ && PPT_ == 8 && H_ <= 2) ? 6 : WAVES_PER_EU;
    // stage parities of the quantity regions: a WENO stage reads the quantities only in its
    // flux phase (its update phase reads the fluxes), so the next stage's quantities can
    // overwrite them after the barrier between the two; a central stencil reads them in
    // the phase that writes the next ones
    static constexpr int QPAR = WENO ? 1 : 2;
};

AT_HD AT_FI int64_t align16(int64_t b) { return (b + 15) & ~int64_t(15); }
AT_HD AT_FI int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }


constexpr int JMAXW = 8;   // row length of the LDS table of extrapolation weights

// LDS layout of a launch (same function on host and device).
//   main region (per PE of the tile: H halo slots, own points, H halo slots)
//   window region (one window of 2*S*H positions per PE boundary), with the
//   quantities double-buffered by stage parity so that stage s+1 of a window
//   is written while stage s is still being read.
template <class C>
struct Layout {
    int64_t EXM, EXW, NW, SOREC;
    int64_t EXR;   // raw staging range [lo - S*H, lo + npts + S*H)
    int64_t o_g, o_glo, o_lam, o_flux, o_gw, o_gwlo, o_lamw, o_fluxw, o_wu, o_wulo, o_wq, o_wR,
        o_SO, o_SOhi, o_pelo, o_keff, o_wt, o_rh, o_rl, total;
    // halo_lds: the scalar FD kind stages the delayed strips of every level in LDS
    AT_HD void init(int npts_max, int npe_max, int jmax, bool halo_lds = false) {
        using L = typename C::lreal;
        const int64_t sl = (int64_t)sizeof(L);
        EXM = npts_max + 2 * C::H * (int64_t)npe_max;
        NW = npe_max + 1;
        EXW = NW * C::WL;
        if (C::HILO) EXW = (EXW + 63) & ~int64_t(63);   // whole wave-sized chunks (direct copy)
        // per PE side: the delayed strips of jmax levels, or (scalar FD kind with the
        // strips in registers) their extrapolation to level n, one level's worth
        const int64_t jl = C::KIND == K_ADR && !halo_lds ? 1 : jmax;
        SOREC = jl * C::S * C::H * C::F;
        // FP32 scalar kind: no raw range (own points go to registers, windows straight
        // into the window region)
        EXR = C::HILO ? 0 : npts_max + 2 * C::S * C::H;
        if (C::F32) EXR = (EXR + 63) & ~int64_t(63);   // whole wave-sized chunks (direct copy)
        const int64_t SR = C::S > 1 ? C::S - 1 : 1;
        int64_t o = 0;
        // the raw range is consumed before the main region is first written
        // (a barrier apart), so the two share the front of the layout
        o_rh = o;    o += align16(C::F * EXR * sl);
        o_rl = o;    o += C::F32 ? align16(C::F * EXR * 4) : 0;
        const int64_t raw_end = o;
        o = 0;
        // main region, two stage parities (a stage reads one, writes the next stage's
        // quantities into the other); the FP32 scalar kind shares its hi part
        // FP32 scalar kind: the lo parts of both stage parities, interleaved (word 2e + parity),
        // at offset 0 of the launch's LDS, so that the own points' stencil reads take
        // their neighbour offsets as instruction immediates; then the hi parts
        if (C::HILO) { o_glo = o; o += align16(2 * EXM * 4); }
        o_g = o;     o += align16((C::HILO ? 1 : C::QPAR) * C::NQ * EXM * sl);
        if (!C::HILO) o_glo = o;
        o_lam = o;   o += C::WENO ? align16(C::QPAR * EXM * sl) : 0;
        o_flux = o;  o += C::WENO ? align16(C::F * EXM * sl) : 0;
        if (o < raw_end) o = raw_end;
        // the scalar FD kind's window quantities are its window state (aliased below)
        o_gw = o;    o += C::KIND == K_ADR ? 0 : align16(C::QPAR * C::NQ * EXW * sl);
        o_gwlo = o;
        o_lamw = o;  o += C::WENO ? align16(C::QPAR * EXW * sl) : 0;
        o_fluxw = o; o += C::WENO ? align16(C::F * EXW * sl) : 0;
        o_wu = o;    o += align16(C::F * EXW * sl);
        o_wulo = o;  o += C::F32 ? align16(C::F * EXW * 4) : 0;
        o_wq = o;    o += align16(2 * C::F * EXW * sl);
        o_wR = o;    o += rk_keeps_stage_rhs<C::S>() ? align16(SR * C::F * EXW * sl) : 0;
        // the strips of the non-scalar kinds arrive by direct copies of 64 words: whole
        // 256-byte chunks
        o_SO = o;    o += align256(2 * (int64_t)npe_max * SOREC * sl);
        o_SOhi = o;  o += C::F32 ? align256(2 * (int64_t)npe_max * jl * C::H * C::F * 4) : 0;
        o_pelo = o;  o += align16((npe_max + 1) * 4);
        o_keff = o;  o += align16(2 * (int64_t)npe_max * 4);
        o_wt = o;    o += C::KIND == K_ADR ? 0 : align16(16 * JMAXW * 8);   // extrapolation weights [k][l]
        total = o;
    }
};

// strip record: FP64: G[s][h][f] doubles; FP32 forms: hi[h][f] floats then lo[s][h][f]
template <class C>
AT_HD AT_FI int64_t record_bytes() {
    return C::F32 ? (int64_t)(C::H * C::F + C::S * C::H * C::F) * 4
                  : (int64_t)C::S * C::H * C::F * 8;
}

// ---------------------------------------------------------------------------
// delays: SplitMix64 finaliser as a counter-based hash
// ---------------------------------------------------------------------------
AT_HD AT_FI uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

constexpr uint64_t GOLDEN = 0x9e3779b97f4a7c15ULL;

// the (seed, problem, step) part of the counter chain: the same for every PE of a step
AT_HD AT_FI uint64_t delay_prefix(const ProbDev& P, int64_t step) {
    const uint64_t z = mix64(P.seed + GOLDEN * (uint64_t)(P.pid + 1));
    return mix64(z + GOLDEN * (uint64_t)(step + 1));
}

// delay of counter (idx, side) given the step's prefix
// (kmax and n_cdf from the uniform copy of the descriptor; the thresholds cdf, indexed
// at run time, from the descriptor in memory, read only for a non-uniform law)
AT_HD AT_FI int draw_delay(const ProbDev& P, const AT_CONST uint64_t* cdf, uint64_t prefix, int64_t idx, int side) {
    const uint64_t z = mix64(prefix + GOLDEN * (uint64_t)(2 * idx + side + 1));
    const uint64_t top = z >> 32;
    if (P.n_cdf == 0) return (int)((top * (uint64_t)(P.kmax + 1)) >> 32);
    int k = 0;
    while (k < P.kmax && top >= cdf[k]) ++k;
    return k;
}

// AT time-extrapolation weights (Sec. 2.2, Table A): Lagrange weights from levels
// -k..-k-J+1 to 0, w_l = prod_{m!=l} (k+m)/(m-l), exact integers, tabulated at compile
// time: WTAB.w[J][k][l], J = 1..JM, k = 0..15.
constexpr int JM = 6;

struct WeightTable {
    double w[JM + 1][16][8];
};
constexpr WeightTable make_weight_table() {
    WeightTable t{};
    for (int J = 1; J <= JM; ++J)
        for (int k = 0; k < 16; ++k)
            for (int l = 0; l < J; ++l) {
                long long num = 1, den = 1;
                for (int m = 0; m < J; ++m) {
                    if (m == l) continue;
                    num *= (long long)(k + m);
                    den *= (long long)(m - l);
                }
                t.w[J][k][l] = (double)(num / den);
            }
    return t;
}
#if defined(__HIPCC__)
__constant__ constexpr WeightTable WTAB = make_weight_table();
#else
constexpr WeightTable WTAB = make_weight_table();
#endif

// ---------------------------------------------------------------------------
// central finite-difference weights (textbook, order 2H)
// ---------------------------------------------------------------------------
template <int H> struct FD;
template <> struct FD<1> {
    AT_HD static constexpr double c1(int o) { return o == 1 ? 0.5 : 0.0; }
    AT_HD static constexpr double c2(int o) { return o == 0 ? -2.0 : 1.0; }
};
template <> struct FD<2> {
    AT_HD static constexpr double c1(int o) { return o == 1 ? 2.0 / 3.0 : -1.0 / 12.0; }
    AT_HD static constexpr double c2(int o) { return o == 0 ? -2.5 : (o == 1 ? 4.0 / 3.0 : -1.0 / 12.0); }
};
template <> struct FD<4> {
    AT_HD static constexpr double c1(int o) {
        return o == 1 ? 0.8 : (o == 2 ? -0.2 : (o == 3 ? 4.0 / 105.0 : -1.0 / 280.0));
    }
    AT_HD static constexpr double c2(int o) {
        return o == 0 ? -205.0 / 72.0 : (o == 1 ? 1.6 : (o == 2 ? -0.2 : (o == 3 ? 8.0 / 315.0 : -1.0 / 560.0)));
    }
};
template <> struct FD<3> {   // unused (WENO); keeps templates well-formed
    AT_HD static constexpr double c1(int) { return 0.0; }
    AT_HD static constexpr double c2(int) { return 0.0; }
};
AT_HD inline double fd_c1(int H, int o) {
    return H == 1 ? FD<1>::c1(o) : H == 2 ? FD<2>::c1(o) : H == 4 ? FD<4>::c1(o) : 0.0;
}
AT_HD inline double fd_c2(int H, int o) {
    return H == 1 ? FD<1>::c2(o) : H == 2 ? FD<2>::c2(o) : H == 4 ? FD<4>::c2(o) : 0.0;
}

// ---------------------------------------------------------------------------
// physics helpers
// ---------------------------------------------------------------------------
template <class R>
AT_HD AT_FI R sq(R x) { return x * x; }

// one-step chemistry, R = 1: T = (gamma-1)(E/rho - u^2/2 - q Y)
AT_HD AT_FI void reactive_prims(const PhysP& P, const double* q, double& rho, double& u, double& T,
                                double& Y) {
    rho = q[0];
    u = q[1] / q[0];
    const double E = q[2] / q[0];
    Y = q[3] / q[0];
    T = (P.gamma - 1.0) * (E - 0.5 * u * u - P.q * Y);
}

AT_HD AT_FI double arrhenius(const PhysP& P, const double* q) {
    double rho, u, T, Y;
    reactive_prims(P, q, rho, u, T, Y);
    return -P.b * rho * Y * exp(-P.ea / T);
}

// Reciprocal: the hardware's approximation (1 ulp) in FP32 on the GPU, a division otherwise.
// fused multiply-add a b + c (one rounding) in either precision
AT_HD AT_FI float fma_r(float a, float b, float c) { return fmaf(a, b, c); }
AT_HD AT_FI double fma_r(double a, double b, double c) { return fma(a, b, c); }
AT_HD AT_FI double rcp_w(double x) { return 1.0 / x; }
AT_HD AT_FI float rcp_w(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// Euler quantities with one reciprocal of rho: u, the pressure and the wave speed |u| + c
template <class Q>
AT_HD AT_FI void euler_uplam(const PhysP& P, const Q* q, Q& u, Q& p, Q& lam) {
    const Q gm = Q(P.gamma);
    const Q ir = Q(1) / q[0];
    u = q[1] * ir;
    p = (gm - Q(1)) * (q[2] - Q(0.5) * q[1] * u);
    lam = fabs(u) + sqrt(gm * p * ir);
}

// reacting Euler quantities of an FP64 state: conserved values g[0..3] (unrounded), fluxes
// g[4..7] and the wave speed.  FP64 for the reciprocal of rho, u and the pressure (a
// difference of large energies); the fluxes and the wave speed in the LDS type LR.
// With src, also the Arrhenius rate -b rho Y exp(-Ea / T), T = p / rho, in FP64.
template <class LR, class G>
AT_HD AT_FI void reul_quant(const PhysP& P, const double* q, G* g, G& lam, LR* src = nullptr) {
    const double ir = 1.0 / q[0];
    const double u = q[1] * ir;
    const double p = (P.gamma - 1.0) * (q[2] - P.q * q[3] - 0.5 * q[1] * u);
    if (src) *src = (LR)(-P.b * q[3] * exp(-P.ea / (p * ir)));
    const LR uf = (LR)u, pf = (LR)p, m = (LR)q[1], en = (LR)q[2], ry = (LR)q[3];
    for (int f = 0; f < 4; ++f) g[f] = (G)q[f];
    g[4] = (G)q[1];
    g[5] = (G)(m * uf + pf);
    g[6] = (G)(uf * (en + pf));
    g[7] = (G)(ry * uf);
    lam = (G)(fabs(uf) + sqrt(LR(P.gamma) * (LR)(p * ir)));
}

// Arrhenius rate -b rho Y exp(-Ea / T) of an FP64 state, T = p / rho
AT_HD AT_FI double arrhenius_p(const PhysP& P, const double* q) {
    const double p = (P.gamma - 1.0) * (q[2] - P.q * q[3] - 0.5 * q[1] * q[1] / q[0]);
    return -P.b * q[3] * exp(-P.ea * q[0] / p);
}

// WENO5-JS reconstruction at the right edge of the middle value v2 of five (candidate
// polynomials p_k on the stencils {v_k, v_k+1, v_k+2}, ideal weights 1/10, 3/5, 3/10,
// nonlinear weights gamma_k / (eps + beta_k)^2 normalised), returned as 6 (vhat - v2).
// In the differences d_ij = v_j - v_i:
//   6 p_k - 6 v2 = r_k:  r_0 = 5 d12 - 2 d01,  r_1 = d12 + 2 d23,  r_2 = 4 d23 - d34
//   beta_k = 13/12 a_k^2 + 1/4 b_k^2 = 13/12 (a_k^2 + 3/13 b_k^2), a_k the second and
//   b_k the first difference of stencil k:  a = (d12 - d01, d23 - d12, d34 - d23),
//   b = (3 d12 - d01, d12 + d23, d34 - 3 d23)
// so that with bh_k = a_k^2 + 3/13 b_k^2 the weights are those of eps at epsh = 12/13 eps.
// FP32: weights gamma_k / (epsh + bh_k)^2 from reciprocals (no overflow of products of
// squares); FP64: the weights multiplied by the three denominators, one division.
// INTERP: the interpolation form (eqs. interpS, fullSten: the candidates' quadratic
// interpolants of the point values half a cell right of v2, ideal weights 1/16, 5/8, 5/16,
// the same smoothness indicators), returned as 8 (vhat - v2):
//   r_0 = 7 d12 - 3 d01,  r_1 = d12 + 3 d23,  r_2 = 5 d23 - d34.
template <class R, bool INTERP = false>
AT_HD AT_FI R weno5_corr(R epsh, R v0, R v1, R v2, R v3, R v4) {
    const R d01 = v1 - v0, d12 = v2 - v1, d23 = v3 - v2, d34 = v4 - v3;
    const R a0 = d12 - d01, a1 = d23 - d12, a2 = d34 - d23;
    const R b0 = R(3) * d12 - d01, b1 = d12 + d23, b2 = d34 - R(3) * d23;
    // e_k = epsh + a_k^2 + (3/13) b_k^2, as two fused multiply-adds after one product
    const R k = R(3.0 / 13.0);
    const R e0 = fma_r(a0, a0, fma_r(k * b0, b0, epsh));
    const R e1 = fma_r(a1, a1, fma_r(k * b1, b1, epsh));
    const R e2 = fma_r(a2, a2, fma_r(k * b2, b2, epsh));
    R r0, r1, r2;
    if constexpr (INTERP) {
        r0 = R(7) * d12 - R(3) * d01;
        r1 = d12 + R(3) * d23;
        r2 = R(5) * d23 - d34;
    } else {
        r0 = R(2) * b0 - d12;
        r1 = d12 + R(2) * d23;
        r2 = d23 - b2;
    }
    // ideal weights in the ratio 1 : 6 : 3 (reconstruction) or 1 : 10 : 5 (interpolation)
    constexpr R g1 = INTERP ? R(10) : R(6), g2 = INTERP ? R(5) : R(3);
    R w0, w1, w2;
    if constexpr (sizeof(R) == 4) {
        w0 = rcp_w(e0 * e0);
        w1 = g1 * rcp_w(e1 * e1);
        w2 = g2 * rcp_w(e2 * e2);
    } else {
        const R s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2;
        w0 = s1 * s2;
        w1 = g1 * (s0 * s2);
        w2 = g2 * (s0 * s1);
    }
    return (w0 * r0 + w1 * r1 + w2 * r2) * rcp_w(w0 + w1 + w2);
}

// ---------------------------------------------------------------------------
// per-thread state (registers on the GPU: every index below is a compile-time
// constant after unrolling)
// ---------------------------------------------------------------------------
template <class C>
struct TS {
    int e[C::PPT];                                // ext index of the own point (-1: none)
    uint32_t eb[C::PPT];                          // FP32 scalar kind: e - H (below 2^16)
    typename C::lreal uh[C::PPT][C::F];           // u^n (FP64 value / FP32 hi)
    float ul[C::PPT][C::F];                       // FP32 lo
    typename C::lreal K[C::S][C::PPT][C::F];      // stage right-hand sides (each dies after its last use)
    typename C::lreal acc[C::PPT][C::F];          // sum_s b_s K_s so far (s ascending)
    float khi[C::PPT];                            // FP32 scalar kind: hi part of K (fixed in a step)
    // reacting Euler kind: Arrhenius rate of the stage state, taken where its quantities are
    typename C::lreal src[C::KIND == K_REUL ? C::PPT : 1];
};

// views of one set of differentiated quantities (main region or one window parity)
template <class C>
struct QV {
    using L = typename C::lreal;
    View<L> g[C::NQ];
    View<float> glo;      // HILO: lo part of g[0]
    View<L> lam;          // WENO: wave speed
    View<L> flux[C::F];   // WENO: interface flux between e and e+1 at e
};

// LDS views of one launch
template <class C>
struct Lds {
    using L = typename C::lreal;
    static constexpr int SR = C::S > 1 ? C::S - 1 : 1;
    QV<C> main[2], win[2];     // main: stage parities
    QV<C> win0;                // FP32 scalar kind: stage-0 window view (lo in wulo)
    View<L> wu[C::F], wq[2][C::F];
    View<float> wulo[C::F];
    View<L> wR[SR][C::F];
    View<L> SO;                // delayed strips [side][level][stage][h][f] (FP32: lo parts);
                               // FP32 scalar kind: halo lo parts extrapolated to level n
    View<float> SOhi;          // FP32 forms: hi parts [side][level][h][f]
    View<int> pelo, keff;
    View<double> wt;           // extrapolation weights w_l(k) at [k * JMAXW + l]
    View<L> rh[C::F];          // raw u^n (FP64 value / FP32 hi) on [lo - S*H, lo + npts + S*H)
    View<float> rl[C::F];      // raw FP32 lo
    int EXM, EXW, SOREC, jmax;
    AT_HD void init(unsigned char* base, const Layout<C>& Lo, int npe_max, int jm, bool halo_lds = false) {
        if (C::KIND == K_ADR && !halo_lds) jm = 1;    // one extrapolated level per side
        EXM = (int)Lo.EXM; EXW = (int)Lo.EXW; SOREC = (int)Lo.SOREC; jmax = jm;
        const int64_t nm = Lo.EXM, nw = Lo.EXW;
        for (int par = 0; par < 2; ++par) {
            const int pg = C::HILO ? 0 : par % C::QPAR, pw = par % C::QPAR;
            for (int q = 0; q < C::NQ; ++q) {
                main[par].g[q] = View<L>{(L*)(base + Lo.o_g) + (pg * C::NQ + q) * nm, nm};
                win[par].g[q] = View<L>{(L*)(base + Lo.o_gw) + (pw * C::NQ + q) * nw, nw};
            }
            // interleaved by parity: the lo part of position e is element 2e of the view
            main[par].glo = View<float>{(float*)(base + Lo.o_glo) + par, C::HILO ? 2 * nm - par : 0};
            main[par].lam = View<L>{(L*)(base + Lo.o_lam) + pw * nm, C::WENO ? nm : 0};
            win[par].glo = View<float>{(float*)(base + Lo.o_gwlo) + par * nw, C::HILO ? nw : 0};
            win[par].lam = View<L>{(L*)(base + Lo.o_lamw) + pw * nw, C::WENO ? nw : 0};
            for (int f = 0; f < C::F; ++f) {
                main[par].flux[f] = View<L>{(L*)(base + Lo.o_flux) + f * nm, C::WENO ? nm : 0};
                win[par].flux[f] = View<L>{(L*)(base + Lo.o_fluxw) + f * nw, C::WENO ? nw : 0};
            }
        }
        for (int f = 0; f < C::F; ++f) {
            wu[f] = View<L>{(L*)(base + Lo.o_wu) + f * nw, nw};
            wulo[f] = View<float>{(float*)(base + Lo.o_wulo) + f * nw, C::F32 ? nw : 0};
            for (int par = 0; par < 2; ++par)
                wq[par][f] = View<L>{(L*)(base + Lo.o_wq) + (par * C::F + f) * nw, nw};
            for (int r = 0; r < SR; ++r)
                wR[r][f] = View<L>{(L*)(base + Lo.o_wR) + (r * C::F + f) * nw,
                                   rk_keeps_stage_rhs<C::S>() ? nw : 0};
        }
        if constexpr (C::KIND == K_ADR) {
            // window quantity g = stage state: FP64 value, or FP32 hi (= raw hi) with lo
            for (int par = 0; par < 2; ++par) {
                if constexpr (C::HILO) {
                    win[par].g[0] = wu[0];
                    win[par].glo = View<float>{(float*)wq[par][0].p, nw};
                } else {
                    win[par].g[0] = wq[par][0];
                }
            }
            // stage 0 of a window is u^n itself: hi in wu, lo in wulo
            win0 = win[0];
            if constexpr (C::HILO) win0.glo = wulo[0];
        }
        // (the padded regions: direct copies write whole 64-word chunks)
        SO = View<L>{(L*)(base + Lo.o_SO), (Lo.o_SOhi - Lo.o_SO) / (int64_t)sizeof(L)};
        SOhi = View<float>{(float*)(base + Lo.o_SOhi), C::F32 ? (Lo.o_pelo - Lo.o_SOhi) / 4 : 0};
        pelo = View<int>{(int*)(base + Lo.o_pelo), npe_max + 1};
        keff = View<int>{(int*)(base + Lo.o_keff), 2 * (int64_t)npe_max};
        wt = View<double>{(double*)(base + Lo.o_wt), C::KIND == K_ADR ? 0 : 16 * JMAXW};
        for (int f = 0; f < C::F; ++f) {
            rh[f] = View<L>{(L*)(base + Lo.o_rh) + f * Lo.EXR, Lo.EXR};
            rl[f] = View<float>{(float*)(base + Lo.o_rl) + f * Lo.EXR, C::F32 ? Lo.EXR : 0};
        }
    }
};

// First item of thread tid in a short work list (a few items per PE) whose items
// are to fill wavefront r of a 256-thread group first, then r+1, ...: a list of
// m items costs ceil(m / 64) wavefront passes instead of one pass in every
// wavefront, and lists of different phases start in different wavefronts.
AT_HD AT_FI int first_item(int tid, int nth, int r) {
    return nth == 256 ? ((tid + 256 - 64 * (r & 3)) & 255) : tid;
}


// compile-time loop: f(std::integral_constant<int, I>) for I in [B, E)
template <int B, int E, class Fn>
AT_HD AT_FI void static_for(Fn&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

AT_HD AT_FI int64_t wrapi(int64_t x, int64_t n) {
    int64_t r = x % n;
    return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------------------
// quantities: differentiated values written at an ext position
// ---------------------------------------------------------------------------
// q: full state at the point (qreal).  For HILO the caller writes hi/lo itself.
// src (reacting Euler kind, may be null): receives the Arrhenius rate of the state
template <class C>
AT_HD AT_FI void put_quant(const QV<C>& L, const PhysP& P, int64_t e, const typename C::qreal* q,
                           typename C::lreal* src = nullptr) {
    using Q = typename C::qreal;
    using LR = typename C::lreal;
    if constexpr (C::KIND == K_ADR) {
        L.g[0][e] = (LR)q[0];
    } else if constexpr (C::KIND == K_WSCAL) {
        L.g[0][e] = (LR)q[0];
        if (P.pde == PDE_BURGERS) {
            L.g[1][e] = (LR)(Q(0.5) * q[0] * q[0]);
            L.lam[e] = (LR)fabs(q[0]);
        } else {
            L.g[1][e] = (LR)(Q(P.c) * q[0]);
            L.lam[e] = (LR)fabs(Q(P.c));
        }
    } else if constexpr (C::KIND == K_EUL) {
        Q u, p, lam;
        euler_uplam<Q>(P, q, u, p, lam);
        for (int f = 0; f < 3; ++f) L.g[f][e] = (LR)q[f];
        L.g[3][e] = (LR)q[1];
        L.g[4][e] = (LR)(q[1] * u + p);
        L.g[5][e] = (LR)(u * (q[2] + p));
        L.lam[e] = (LR)lam;
    } else if constexpr (C::KIND == K_REUL) {
        double qd[4] = {(double)q[0], (double)q[1], (double)q[2], (double)q[3]};
        LR g[8], lam;
        reul_quant<LR, LR>(P, qd, g, lam, src);
        for (int j = 0; j < 8; ++j) L.g[j][e] = g[j];
        L.lam[e] = lam;
    } else {  // K_RNS
        double qd[4] = {(double)q[0], (double)q[1], (double)q[2], (double)q[3]};
        double rho, u, T, Y;
        reactive_prims(P, qd, rho, u, T, Y);
        const double p = rho * T;
        // flux form: C1..C4, u, T, Y; chain rule: the primitives rho, u, p, T, Y (slots
        // 5, 6 unused), chosen value by value (one store per slot)
        const bool ch = P.form != 0;
        L.g[0][e] = (LR)(ch ? rho : qd[1]);
        L.g[1][e] = (LR)(ch ? u : qd[1] * u + p);
        L.g[2][e] = (LR)(ch ? p : u * (qd[2] + p));
        L.g[3][e] = (LR)(ch ? T : qd[3] * u);
        L.g[4][e] = (LR)(ch ? Y : u);
        if (!ch) {
            L.g[5][e] = (LR)T;
            L.g[6][e] = (LR)Y;
        }
    }
}

// quantity values (qreal) of a state, without writing LDS: used by the halo fill
template <class C>
AT_HD AT_FI void quant_values(const PhysP& P, const typename C::qreal* q, typename C::qreal* g,
                              typename C::qreal& lam) {
    using Q = typename C::qreal;
    if constexpr (C::KIND == K_ADR) {
        g[0] = q[0];
        lam = Q(0);
    } else if constexpr (C::KIND == K_WSCAL) {
        g[0] = q[0];
        if (P.pde == PDE_BURGERS) { g[1] = Q(0.5) * q[0] * q[0]; lam = fabs(q[0]); }
        else { g[1] = Q(P.c) * q[0]; lam = fabs(Q(P.c)); }
    } else if constexpr (C::KIND == K_EUL) {
        Q u, p;
        euler_uplam<Q>(P, q, u, p, lam);
        g[0] = q[0]; g[1] = q[1]; g[2] = q[2];
        g[3] = q[1]; g[4] = q[1] * u + p; g[5] = u * (q[2] + p);
    } else if constexpr (C::KIND == K_REUL) {
        double qd[4] = {(double)q[0], (double)q[1], (double)q[2], (double)q[3]};
        reul_quant<typename C::lreal, Q>(P, qd, g, lam);
    } else {
        double qd[4] = {(double)q[0], (double)q[1], (double)q[2], (double)q[3]};
        double rho, u, T, Y;
        reactive_prims(P, qd, rho, u, T, Y);
        const double p = rho * T;
        const bool ch = P.form != 0;   // chain rule: the primitives (slots 5, 6 unused)
        g[0] = ch ? rho : qd[1];
        g[1] = ch ? u : qd[1] * u + p;
        g[2] = ch ? p : u * (qd[2] + p);
        g[3] = ch ? T : qd[3] * u;
        g[4] = ch ? Y : u;
        g[5] = ch ? 0.0 : T;
        g[6] = ch ? 0.0 : Y;
        lam = Q(0);
    }
}

// ---------------------------------------------------------------------------
// right-hand side at ext position e
// ---------------------------------------------------------------------------
template <class C>
AT_HD AT_FI typename C::lreal d1(const View<typename C::lreal>& g, int64_t e) {
    using LR = typename C::lreal;
    LR s = LR(FD<C::H>::c1(1)) * (g[e + 1] - g[e - 1]);
    for (int o = 2; o <= C::H; ++o) s += LR(FD<C::H>::c1(o)) * (g[e + o] - g[e - o]);
    return s;
}

template <class C>
AT_HD AT_FI typename C::lreal d2(const View<typename C::lreal>& g, int64_t e) {
    using LR = typename C::lreal;
    LR s = LR(FD<C::H>::c2(0)) * g[e];
    for (int o = 1; o <= C::H; ++o) s += LR(FD<C::H>::c2(o)) * (g[e + o] + g[e - o]);
    return s;
}

// Build option: the own points' interface fluxes of the FP32 WENO kinds take the
// neighbour values from adjacent lanes (DPP wave shifts; lanes hold consecutive points)
// instead of LDS reads, with LDS reads where a neighbour lies past a wave or PE edge.  Off
// by default: the shifts are VALU instructions in a VALU-bound phase, and it measured
// slower than the LDS reads.
#ifndef AT_WENO_DPP
#define AT_WENO_DPP 0
#endif
#if AT_WENO_DPP && defined(__HIP_DEVICE_COMPILE__)
constexpr bool WENO_DPP = true;
__device__ __forceinline__ float lane_prev(float v) {   // the value of lane - 1 (wave_shr:1)
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float lane_next(float v) {   // the value of lane + 1 (wave_shl:1)
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, false));
}
#else
constexpr bool WENO_DPP = false;
inline float lane_prev(float v) { return v; }
inline float lane_next(float v) { return v; }
#endif

// WENO interface flux between e and e+1 (local Lax-Friedrichs splitting), kept as
// twice the flux: with v+ = C + al Q on e-2..e+2 and v- = C - al Q on e+3..e-1,
//   2 F = v+_e + v-_{e+1} + (corr(v+) + corr(v-)) / 6      (reconstruction)
//   2 F = v+_e + v-_{e+1} + (corr(v+) + corr(v-)) / 8      (interpolation form)
// (the split fluxes are (C +- al Q) / 2; their smoothness indicators scale by 4, so the
// weights take 4 epsh)
// LANES (build option above): the neighbours of an interior point from adjacent lanes.
// INTERP: the interpolation form (the corrections are 8 (vhat - v2) there).
template <class C, bool LANES, bool INTERP>
AT_HD AT_FI void iface_flux_form(const QV<C>& L, const PhysP& P, int64_t e, bool interior) {
    using LR = typename C::lreal;
    const LR a0 = L.lam[e], a1 = L.lam[e + 1];
    const LR al = a0 > a1 ? a0 : a1;
    const LR eps = C::F32 ? LR(P.epswf) : LR(P.epsw);
#pragma unroll
    for (int f = 0; f < C::F; ++f) {
        const View<LR>& Q = L.g[f];
        const View<LR>& Cf = L.g[C::F + f];
        LR q[6], c[6];
        if constexpr (LANES) {   // neighbours e-2..e+3 from lanes -2..+3 (interior points)
            q[2] = Q[e];
            c[2] = Cf[e];
            q[1] = lane_prev(q[2]); q[0] = lane_prev(q[1]);
            q[3] = lane_next(q[2]); q[4] = lane_next(q[3]); q[5] = lane_next(q[4]);
            c[1] = lane_prev(c[2]); c[0] = lane_prev(c[1]);
            c[3] = lane_next(c[2]); c[4] = lane_next(c[3]); c[5] = lane_next(c[4]);
        }
        if (!LANES || !interior) {
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                q[m] = Q[e - 2 + m];
                c[m] = Cf[e - 2 + m];
            }
        }
        LR vp[5], vm[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            vp[m] = c[m] + al * q[m];
            vm[m] = c[5 - m] - al * q[5 - m];
        }
        const LR cp = weno5_corr<LR, INTERP>(eps, vp[0], vp[1], vp[2], vp[3], vp[4]);
        const LR cm = weno5_corr<LR, INTERP>(eps, vm[0], vm[1], vm[2], vm[3], vm[4]);
        L.flux[f][e] = (vp[2] + vm[2]) + (cp + cm) * LR(INTERP ? 1.0 / 8.0 : 1.0 / 6.0);
    }
}

// K at ext position e; q = the point's own state (qreal) for sources / primitives
// FP32 scalar FD kind: -c u_x + alpha u_xx (+ r u (1 - u)) at ext position e whose own
// hi and lo values hc, lc the caller holds (they equal the region's values at e), as
// one central stencil on differences to the centre (the weights of each derivative sum
// to zero), hi and lo differences taken separately (hi - hi exact for neighbouring values)
template <class C>
AT_HD AT_FI float rhs_adr_hilo(const QV<C>& L, const PhysP& P, int64_t e, float hc, float lc) {
    // every LDS read first (adjacent positions, so that they pair), then the arithmetic
    float hp[C::H], hm[C::H], lp[C::H], lm[C::H];
#pragma unroll
    for (int o = 1; o <= C::H; ++o) {
        hm[o - 1] = L.g[0][e - o];
        lm[o - 1] = L.glo[e - o];
        hp[o - 1] = L.g[0][e + o];
        lp[o - 1] = L.glo[e + o];
    }
    float k = 0.f;
#pragma unroll
    for (int o = 1; o <= C::H; ++o) {
        const float dp = (hp[o - 1] - hc) + (lp[o - 1] - lc);
        const float dm = (hm[o - 1] - hc) + (lm[o - 1] - lc);
        k += P.lpf[o - 1] * dp;
        k += P.lmf[o - 1] * dm;
    }
    if (P.pde == PDE_ADR_LOGISTIC) {
        const float u = hc + lc;
        k += P.rf * u * (1.f - u);
    }
    return k;
}

// FP32 scalar FD kind at an own point whose hi and lo parts the caller holds:
//   K = khi + sum_o (lpf_o l_{e+o} + lmf_o l_{e-o}) - c0 l_e + r u (1 - u),  u = h_e + l_e,
// where khi = sum_o lpf_o (h_{e+o} - h_e) + lmf_o (h_{e-o} - h_e) is the hi parts' share, fixed
// within a step (the hi parts do not change), and the lo parts l are those of the stage.
// The stencil's weights sum to zero, so this is the stencil of h + l; the lo parts are
// the small stage increments and compensations, so their products need no difference form.
// lo2: the interleaved lo parts (element 2e + parity); eb = e - H >= 0, so every neighbour is
// at a non-negative offset from element 2 eb.
// Returns the neighbours' share sum_o (lpf_o l_{e+o} + lmf_o l_{e-o}); lc receives l_e.
template <class C>
AT_HD AT_FI float hilo_lo_sum(const View<float>& lo2, uint32_t eb, int par, const PhysP& P, float& lc) {
    float v[2 * C::H + 1];
#pragma unroll
    for (int j = 0; j <= 2 * C::H; ++j) v[j] = lo2[2 * (int64_t)(eb + (uint32_t)j) + par];
    lc = v[C::H];
    float k = 0.f;
#pragma unroll
    for (int o = C::H; o >= 1; --o) {
        k = fmaf(P.lmf[o - 1], v[C::H - o], k);
        k = fmaf(P.lpf[o - 1], v[C::H + o], k);
    }
    return k;
}

// src (reacting Euler kind, may be null): the Arrhenius rate of q, taken with its quantities
template <class C>
AT_HD AT_FI void rhs_at(const QV<C>& L, const PhysP& P, int64_t e, const typename C::qreal* q,
                        typename C::lreal* K, const typename C::lreal* src = nullptr) {
    using LR = typename C::lreal;
    if constexpr (C::KIND == K_ADR) {
        // -c u_x + alpha u_xx as one central stencil on differences to the centre
        // (the weights of each derivative sum to zero)
        if constexpr (C::HILO) {
            // windows only (the main region's lo parts are interleaved by parity)
            K[0] = rhs_adr_hilo<C>(L, P, e, L.g[0][e], L.glo[e]);
        } else {
            const LR uc = L.g[0][e];
            LR k = LR(0);
#pragma unroll
            for (int o = 1; o <= C::H; ++o) {
                k += LR(P.lp[o - 1]) * (L.g[0][e + o] - uc);
                k += LR(P.lm[o - 1]) * (L.g[0][e - o] - uc);
            }
            if (P.pde == PDE_ADR_LOGISTIC) k += LR(P.r) * (LR)q[0] * (LR(1) - (LR)q[0]);
            K[0] = k;
        }
    } else if constexpr (C::KIND == K_RNS) {
        const LR idx = LR(P.inv_dx), idx2 = LR(P.inv_dx2);
        double qd[4] = {(double)q[0], (double)q[1], (double)q[2], (double)q[3]};
        double rho, u, T, Y;
        reactive_prims(P, qd, rho, u, T, Y);
        if (P.form) {
            // chain rule (Sec. 4 after eq. convEq): the convective products differentiated
            // through the primitives rho, u, p, Y, e.g. (rho u Y)_x = rho u Y_x + rho u_x Y
            // + rho_x u Y; rho E = p/(gamma-1) + rho u^2/2 + q rho Y
            const LR rx = d1<C>(L.g[0], e) * idx, ux = d1<C>(L.g[1], e) * idx;
            const LR px = d1<C>(L.g[2], e) * idx, Yx = d1<C>(L.g[4], e) * idx;
            const LR uxx = d2<C>(L.g[1], e) * idx2, Txx = d2<C>(L.g[3], e) * idx2;
            const LR Yxx = d2<C>(L.g[4], e) * idx2;
            const LR r = LR(rho), uu = LR(u), YY = LR(Y), pp = LR(rho * T), rE = LR(qd[2]);
            const LR mu43 = LR(4.0 / 3.0) * LR(P.mu);
            const LR dE = px * LR(1.0 / (P.gamma - 1.0)) + LR(0.5) * rx * uu * uu + r * uu * ux +
                          LR(P.q) * (rx * YY + r * Yx);
            K[0] = -(rx * uu + r * ux);
            K[1] = -(rx * uu * uu + LR(2) * r * uu * ux + px) + mu43 * uxx;
            K[2] = -(ux * (rE + pp) + uu * (dE + px)) + mu43 * (ux * ux + uu * uxx) + LR(P.kappa) * Txx +
                   LR(P.q * P.rhoD) * Yxx;
            K[3] = -(r * uu * Yx + r * ux * YY + rx * uu * YY) + LR(P.rhoD) * Yxx + LR(arrhenius(P, qd));
            return;
        }
        const LR ux = d1<C>(L.g[4], e) * idx, uxx = d2<C>(L.g[4], e) * idx2;
        const LR Txx = d2<C>(L.g[5], e) * idx2, Yxx = d2<C>(L.g[6], e) * idx2;
        const LR mu43 = LR(4.0 / 3.0) * LR(P.mu);
        K[0] = -(d1<C>(L.g[0], e) * idx);
        K[1] = -(d1<C>(L.g[1], e) * idx) + mu43 * uxx;
        K[2] = -(d1<C>(L.g[2], e) * idx) + mu43 * (ux * ux + LR(u) * uxx) + LR(P.kappa) * Txx +
               LR(P.q * P.rhoD) * Yxx;
        K[3] = -(d1<C>(L.g[3], e) * idx) + LR(P.rhoD) * Yxx + LR(arrhenius(P, qd));
    } else {  // WENO kinds
        const LR hidx = C::F32 ? LR(P.hidxf) : LR(P.hidx);    // the fluxes are kept doubled
#pragma unroll
        for (int f = 0; f < C::F; ++f) K[f] = -((L.flux[f][e] - L.flux[f][e - 1]) * hidx);
        if constexpr (C::KIND == K_REUL) {
            if (src) {
                K[3] += *src;
            } else {
                double qd[4] = {(double)q[0], (double)q[1], (double)q[2], (double)q[3]};
                K[3] += LR(arrhenius_p(P, qd));
            }
        }
        if constexpr (C::KIND == K_WSCAL) {
            if (P.pde == PDE_ADR_LOGISTIC) K[0] += LR(P.r) * (LR)q[0] * (LR(1) - (LR)q[0]);
        }
    }
}

// ---------------------------------------------------------------------------
// non-periodic ends (reactive NS kind): the points whose interior stencil would leave
// the domain.  The two end points take second-order one-sided differences and the
// characteristic (LODI) form of the convective terms with the incoming waves removed
// (non-reflecting conditions); the others second-order central differences.  The
// arithmetic is FP64 in every form.  x: global index of the point, e its ext position;
// every point read lies inside the domain (the first and the last PE hold at least four).
// ---------------------------------------------------------------------------
template <class C>
AT_HD AT_FI void end_prims(const QV<C>& L, int64_t e, double* v) {
    // rho, u, p, T, Y from C1 = rho u, C2 = rho u^2 + p, u, T, Y
    const double u = (double)L.g[4][e], T = (double)L.g[5][e];
    const double p = (double)L.g[1][e] - (double)L.g[0][e] * u;
    v[0] = p / T;
    v[1] = u;
    v[2] = p;
    v[3] = T;
    v[4] = (double)L.g[6][e];
}

template <class C>
AT_HD AT_FI void rhs_end_rns(const QV<C>& L, const PhysP& P, int64_t e, int64_t x, int64_t N, const double* q,
                             typename C::lreal* K) {
    using LR = typename C::lreal;
    const double idx = P.inv_dx, idx2 = P.inv_dx2;
    double cv[4], ux, uxx, Txx, Yxx, uc;
    if (x == 0 || x == N - 1) {
        const int sg = x == 0 ? 1 : -1;
        double f[4][5];
        for (int m = 0; m < 4; ++m) end_prims<C>(L, e + sg * m, f[m]);
        double d1v[5], d2v[5];
        for (int v = 0; v < 5; ++v) {
            d1v[v] = (double)sg * (4.0 * f[1][v] - 3.0 * f[0][v] - f[2][v]) * (0.5 * idx);
            d2v[v] = (2.0 * f[0][v] - 5.0 * f[1][v] + 4.0 * f[2][v] - f[3][v]) * idx2;
        }
        const double rho = f[0][0], u = f[0][1], p = f[0][2], Y = f[0][4];
        const double c = sqrt(P.gamma * p / rho);
        double L1 = (u - c) * (d1v[2] - rho * c * d1v[1]);
        double L2 = u * (c * c * d1v[0] - d1v[2]);
        double L3 = u * d1v[4];
        double L5 = (u + c) * (d1v[2] + rho * c * d1v[1]);
        // a wave entering the domain (speed > 0 at the left end, < 0 at the right) is removed
        const double sgn = (double)sg;
        if (sgn * (u - c) > 0.0) L1 = 0.0;
        if (sgn * u > 0.0) { L2 = 0.0; L3 = 0.0; }
        if (sgn * (u + c) > 0.0) L5 = 0.0;
        const double d1 = (L2 + 0.5 * (L5 + L1)) / (c * c);
        const double d2 = 0.5 * (L5 + L1);
        const double d3 = (L5 - L1) / (2.0 * rho * c);
        cv[0] = -d1;
        cv[1] = -(u * d1 + rho * d3);
        cv[3] = -(Y * d1 + rho * L3);
        cv[2] = -(0.5 * u * u * d1 + d2 / (P.gamma - 1.0) + rho * u * d3) + P.q * cv[3];
        ux = d1v[1];
        uxx = d2v[1];
        Txx = d2v[3];
        Yxx = d2v[4];
        uc = u;
    } else {
        for (int f = 0; f < 4; ++f) cv[f] = -((double)L.g[f][e + 1] - (double)L.g[f][e - 1]) * (0.5 * idx);
        const double um = L.g[4][e - 1], u0 = L.g[4][e], up = L.g[4][e + 1];
        ux = (up - um) * (0.5 * idx);
        uxx = (up - 2.0 * u0 + um) * idx2;
        Txx = ((double)L.g[5][e + 1] - 2.0 * (double)L.g[5][e] + (double)L.g[5][e - 1]) * idx2;
        Yxx = ((double)L.g[6][e + 1] - 2.0 * (double)L.g[6][e] + (double)L.g[6][e - 1]) * idx2;
        uc = u0;
    }
    const double mu43 = (4.0 / 3.0) * P.mu;
    K[0] = LR(cv[0]);
    K[1] = LR(cv[1] + mu43 * uxx);
    K[2] = LR(cv[2] + mu43 * (ux * ux + uc * uxx) + P.kappa * Txx + P.q * P.rhoD * Yxx);
    K[3] = LR(cv[3] + P.rhoD * Yxx + arrhenius(P, q));
}

// ---------------------------------------------------------------------------
// global memory helpers
// ---------------------------------------------------------------------------
template <class C>
AT_HD AT_FI GView<typename C::lreal> st_view(const ProbDev& P, int which) {
    return GView<typename C::lreal>{(typename C::lreal*)(which ? P.st_hi[1] : P.st_hi[0]), (int64_t)C::F * P.n};
}
AT_HD AT_FI GView<float> lo_view(const ProbDev& P, int which, bool f32) {
    return GView<float>{(float*)(which ? P.st_lo[1] : P.st_lo[0]), f32 ? (int64_t)P.F * P.n : 0};
}


// ---------------------------------------------------------------------------
// the tile step
//
//   P1  every global read in one phase: the raw range [lo - S*H, lo + npts + S*H)
//       of u^n, PE offsets, delays, delayed strips of the ring -> LDS
//   P2  own points (registers, stage-s0 quantities), boundary windows of level n
//       from the raw range (stage-0 quantities, ring records of stage 0)
//   per stage s:  A  own quantities of V(s), halo fill (extrapolated strips, or
//                    the window's synchronous stage s when the delay is 0)
//                 B  [WENO: interface fluxes]  K_s at own points; R_s on the
//                    windows and their synchronous stage s+1 (+ ring record)
//   P5  u^{n+1} (or K_s to the workspace in per-stage mode)
// ---------------------------------------------------------------------------
template <class C>
AT_HD AT_FI int64_t ring_lo_off(int s, int h, int f) { return (int64_t)C::H * C::F + ((int64_t)s * C::H + h) * C::F + f; }

// STEP: the launch is a whole step (stages 0..S-1, no stage inputs or outputs), so the
// stage range is known at compile time; otherwise it is read from the arguments.
// STAGED (scalar FD kind, run option halo_lds): the delayed strips staged in LDS instead
// of registers; a kernel of its own, so that the default kernel carries none of its code.
template <class C, bool STEP, bool STAGED, class RT>
AT_HD void tile_step(RT& rt, const KArgs& a, const Tile& t_in, const AT_CONST ProbDev& P_in, int64_t n_in,
                     unsigned char* lds_base) {
    const ProbDev P = uniform_copy(P_in);
    using LR = typename C::lreal;
    using Q = typename C::qreal;
    constexpr int F = C::F, H = C::H, S = C::S, PPT = C::PPT, WL = C::WL, NQ = C::NQ;

    // tile and problem scalars, once per tile, uniform (scalar registers on the GPU)
    Tile t;
    t.prob = uni(t_in.prob);
    t.pe0 = uni(t_in.pe0);
    t.npe = uni(t_in.npe);
    t.npts = uni(t_in.npts);
    t.lo = uni(t_in.lo);
    const int64_t n = uni(n_in);
    PhysP PP;
    PP.pde = uni(P.pde);
    PP.interp = uni(P.interp);
    PP.form = uni(P.form);
    PP.c = uni(P.c); PP.alpha = uni(P.alpha); PP.r = uni(P.r); PP.gamma = uni(P.gamma);
    PP.q = uni(P.q); PP.ea = uni(P.ea); PP.b = uni(P.b); PP.mu = uni(P.mu);
    PP.kappa = uni(P.kappa); PP.rhoD = uni(P.rhoD); PP.eps = uni(P.eps);
    PP.inv_dx = uni(P.inv_dx); PP.inv_dx2 = uni(P.inv_dx2); PP.dt = uni(P.dt);
    PP.cf = uni(P.cf); PP.alphaf = uni(P.alphaf); PP.rf = uni(P.rf);
    PP.inv_dxf = uni(P.inv_dxf); PP.inv_dx2f = uni(P.inv_dx2f);
    PP.dtf = uni(P.dtf);
    PP.epsw = uni(PP.eps * (48.0 / 13.0));
    PP.hidx = uni(0.5 * PP.inv_dx);
    PP.epswf = uni((float)PP.epsw);
    PP.hidxf = uni((float)PP.hidx);
    PP.c0f = uni(P.c0f);
    PP.rlf = uni(P.rlf);
    if constexpr (C::KIND == K_ADR) {
        for (int o = 0; o < H; ++o) {
            PP.lp[o] = uni(P.lin_p[o]); PP.lm[o] = uni(P.lin_m[o]);
            PP.lpf[o] = uni(P.lpf[o]); PP.lmf[o] = uni(P.lmf[o]);
        }
    }
    // memory of the problem (uniform)
    const int64_t Pp = uni((int64_t)P.p);
    const int Dring = uni(P.D);
    const int64_t recb = uni(P.rec_bytes);
    unsigned char* const ring = (unsigned char*)uni((int64_t)(uintptr_t)P.ring);
    using TB = RKTab<S>;

    // LDS layout sized by this tile (the launch allocates the largest over its tiles)
    // scalar FD kind: the delayed strips staged in LDS (run option) instead of registers
    constexpr bool staged = STAGED && C::KIND == K_ADR;
    AT_CHECK(staged == (C::KIND == K_ADR && (a.flags & KF_HALO_LDS) != 0), "halo staging", staged, a.flags);
    Layout<C> Lo;
    Lo.init(t.npts, t.npe, a.jmax, staged);
    AT_CHECK(Lo.total <= a.lds_bytes, "tile LDS", Lo.total, a.lds_bytes);
    Lds<C> L;
    L.init(lds_base, Lo, t.npe, a.jmax, staged);


    const int nth = rt.nthreads();
    const int s0 = STEP ? 0 : a.s_begin, s1 = STEP ? S - 1 : a.s_end;
    const bool first = STEP || s0 == 0;
    const bool stage_io = !STEP && (a.flags & KF_STAGE_IO) != 0;
    AT_CHECK(!STEP || (a.s_begin == 0 && a.s_end == S - 1 && !(a.flags & KF_STAGE_IO)), "whole step",
             a.s_begin, a.s_end);
    const int cur = (int)(n & 1), nxt = cur ^ 1;
    const GView<LR> st = st_view<C>(P, cur);
    const GView<float> stlo = lo_view(P, cur, C::F32);
    const bool use_lo = C::F32 && P.keep_lo;
    const int64_t N = uni(P.n);
    const int J = uni(P.J);
    const LR dt = C::F32 ? LR(PP.dtf) : LR(PP.dt);
    AT_CHECK(t.npts <= a.npts_max && t.npe <= a.npe_max, "tile size", t.npts, a.npts_max);
    AT_CHECK(J <= a.jmax && J <= JM, "jmax", J, a.jmax);
    AT_CHECK(t.npts <= nth * PPT, "points per thread", t.npts, nth * PPT);

    // strip ring: slot of level n (levels n - d, 0 <= d < D, are slot_n - d mod D),
    // records of the tile's PEs at a slot are 2 * npe consecutive records
    const int slot_n = uni((int)(n % Dring));
    // ring element offsets (in 4-byte words from the ring base; the ring is under 4 GiB)
    const uint32_t slot_stride_w = (uint32_t)(Pp * 2 * recb / 4);
    const uint32_t recw = (uint32_t)(recb / 4);
    const uint32_t ring_tile_w = (uint32_t)((int64_t)t.pe0 * 2 * recb / 4);
    const float* const ring_f = (const float*)ring;
    // first word of the record of PE (t.pe0 + k), side, at level n - d
    auto rec_back = [&](int d, int k, int side) -> uint32_t {
        AT_CHECK(d >= 0 && d < Dring, "ring depth", d, Dring);
        int slot = slot_n - d;
        if (slot < 0) slot += Dring;
        const int64_t idx = ((int64_t)slot * Pp + t.pe0 + k) * 2 + side;
        AT_CHECK(idx >= 0 && idx < (int64_t)Dring * Pp * 2, "ring record", idx, (int64_t)Dring * Pp * 2);
        return ring_tile_w + (uint32_t)slot * slot_stride_w + (uint32_t)(2 * k + side) * recw;
    };
    const uint32_t ring_n_w = ring_tile_w + (uint32_t)slot_n * slot_stride_w;
    // ring record of PE (t.pe0 + k), side, level n: stage s at halo point h
    auto rec_store = [&](int k, int side, int s, int h, int f, LR v, float hi) {
        AT_CHECK(k >= 0 && k < t.npe, "ring store", k, t.npe);
        const uint32_t w0 = ring_n_w + (uint32_t)(2 * k + side) * recw;
        if constexpr (C::F32) {
            gst((float*)ring, w0 + (uint32_t)ring_lo_off<C>(s, h, f), (float)v);
            if (s == 0) gst((float*)ring, w0 + (uint32_t)(h * F + f), hi);
        } else {
            gst((double*)ring, w0 / 2 + (uint32_t)(((int64_t)s * H + h) * F + f), (double)v);
        }
    };
    // write the window's synchronous-stage strip value at window position w of boundary b
    auto strip_out = [&](int b, int w, int s, int f, LR v, float hi) {
        const int h2 = w - (S - 1) * H;
        if (h2 < 0 || h2 >= 2 * H) return;
        if (h2 < H) {                       // left halo of PE b
            if (b < t.npe) rec_store(b, 0, s, h2, f, v, hi);
        } else {                            // right halo of PE b-1
            if (b >= 1) rec_store(b - 1, 1, s, h2 - H, f, v, hi);
        }
    };

    // delay of PE (t.pe0 + k), side: drawn and effective (clamped to the held history)
    const uint64_t dprefix = uni((int64_t)delay_prefix(P, n));
    auto delays_of = [&](int k, int side, int& kd) -> int {
        const int64_t pe = t.pe0 + k;
        if (P.ov && n >= P.ov_step0 && n < P.ov_step0 + P.ov_n) {
            const int64_t oi = ((n - P.ov_step0) * P.p + pe) * 2 + side;
            AT_CHECK(oi >= 0 && oi < P.ov_n * P.p * 2, "override", oi, P.ov_n * P.p * 2);
            kd = gld(P.ov, (uint32_t)oi);
            // consumed here, so that no later join of the paths waits for the vector-memory
            // counter (which would also wait for the tile's direct copies in flight)
            vm_drain();
        } else if (P.gran == G_PE) {
            kd = draw_delay(P, P_in.cdf, dprefix, pe, 0);
        } else if (P.gran == G_PE_SIDE) {
            kd = draw_delay(P, P_in.cdf, dprefix, pe, side);
        } else {
            kd = draw_delay(P, P_in.cdf, dprefix, side == 0 ? pe : (pe + 1 == P.p ? 0 : pe + 1), 0);
        }
        int ke;
        if (P.mode == M_AT) {
            ke = kd;
            if ((int64_t)ke > n - (J - 1)) ke = (int)(n - (J - 1));
            if (ke < 0) ke = 0;
        } else if (P.mode == M_AS) {
            ke = (int64_t)kd < n ? kd : (int)n;
        } else {
            ke = 0;
        }
        return ke;
    };

    // ---- P1: every global read of the tile in one phase -----------------------------
    //   raw u^n on [lo - S*H, lo + npts + S*H) (own points and boundary windows),
    //   PE offsets, delays, delayed strips of the ring, stage inputs (per-stage mode)
    constexpr int SH = S * H;
    // floor(p N / P), the first point of PE p, from the planner's table
    const GView<const int32_t> peoff{P.peoff, Pp + 1};
    auto pe_offset = [&](int64_t pe) -> int64_t { return (int64_t)peoff.ld(pe); };
    constexpr int nrec = S * H * F;              // lo (FP32) or value (FP64) words of a level
    constexpr int nhi = C::F32 ? H * F : 1;      // FP32 hi words of a level
    // FP32 forms: the raw range is copied into LDS directly (no registers), and all
    // levels of the first PE side are loaded before it is waited for; FP64: the raw
    // range goes through registers, and one level (the records take twice the
    // registers) is loaded before it is stored
    constexpr bool RAW_DMA = C::F32;
    // FP32 scalar kind: no raw range; own points are loaded into registers and the
    // boundary windows copied straight into the window region, so that the own-point
    // and window set-up needs no phase (and barrier) of its own
    constexpr bool OWN_REG = C::HILO;
    constexpr int JPF = C::F32 ? (JM < 3 ? JM : 3) : 1;
    constexpr int JPR = JPF > 0 ? JPF : 1;
    // delays of a PE side (into LDS, and the log); the number of ring levels it reads
    auto side_delays = [&](int side_idx, int& ke) -> int {
        const int k = side_idx >> 1, side = side_idx & 1;
        int kd;
        ke = delays_of(k, side, kd);
        L.keff[side_idx] = ke;
        if ((a.flags & KF_LOG) && first && P.log_drawn) {
            const int64_t li = (wrapi(n, P.log_cap) * P.p + t.pe0 + k) * 2 + side;
            AT_CHECK(li >= 0 && li < P.log_cap * P.p * 2, "log", li, P.log_cap * P.p * 2);
            gst(P.log_drawn, (uint32_t)li, (uint8_t)kd);
            gst(P.log_eff, (uint32_t)li, (uint8_t)ke);
        }
        // delayed strips (and level n in per-stage mode) from the ring
        return ke == 0 ? (first ? 0 : 1) : J;
    };
    auto ring_ld = [&](int side_idx, int ke, int l, LR (&v)[nrec], float (&vh)[nhi]) {
        const uint32_t w0 = rec_back(ke + l, side_idx >> 1, side_idx & 1);
        if constexpr (C::F32 && (H * F + nrec) % 2 == 0) {
            // an even number of words: every record is 8-byte aligned (the ring base is
            // 256-byte aligned), so the record is read as 64-bit words
            constexpr int nw = H * F + nrec;
#pragma unroll
            for (int j = 0; j < nw / 2; ++j) {
                const uint64_t d = gld((const uint64_t*)ring_f, w0 / 2 + (uint32_t)j);
                const float w[2] = {__builtin_bit_cast(float, (uint32_t)d),
                                    __builtin_bit_cast(float, (uint32_t)(d >> 32))};
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int r = 2 * j + u;
                    if (r < H * F) vh[r < H * F ? r : 0] = w[u];
                    else v[r >= H * F ? r - H * F : 0] = w[u];
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < nrec; ++r) {
                if constexpr (C::F32) v[r] = gld(ring_f, w0 + (uint32_t)(H * F + r));
                else v[r] = gld((const double*)ring_f, w0 / 2 + (uint32_t)r);
            }
            if constexpr (C::F32) {
#pragma unroll
                for (int r = 0; r < H * F; ++r) vh[r] = gld(ring_f, w0 + (uint32_t)r);
            }
        }
    };
    // the delayed strips of every PE side and level (non-scalar kinds): word-wise direct
    // copies of wave-sized chunks of consecutive LDS words, the lo parts (FP64: the
    // values) into SO [side][level][word], the FP32 hi parts into SOhi [side][level][word].
    // Each lane takes its PE side's delay from the counter-based draw itself; a level the
    // side does not read copies the side's nearest record (unused).  Lanes past the end
    // copy the last word again into the chunk's padding.
    auto ring_copy = [&](int tid) {
        const int lane = tid & 63, jm = L.jmax;
        auto rec_word = [&](int p, int wpl) -> uint32_t {   // ring word of LDS word p
            const int per_side = jm * wpl;
            const int side_idx = p / per_side, rem = p - side_idx * per_side;
            const int l = rem / wpl, r = rem - l * wpl;
            int kd;
            const int ke = delays_of(side_idx >> 1, side_idx & 1, kd);
            const int jeff = ke == 0 ? (first ? 0 : 1) : J;
            const int lv = l < jeff ? l : 0;
            return rec_back(ke + lv, side_idx >> 1, side_idx & 1) + (uint32_t)r;
        };
        constexpr int wlo = C::F32 ? nrec : 2 * nrec;         // SO words of a level
        const int nso = 2 * t.npe * jm * wlo;
        float* const so = (float*)&L.SO[0];
        for (int c = tid & ~63; c < nso; c += nth) {
            AT_CHECK((int64_t)(c + 64) * 4 <= L.SO.n * (int64_t)sizeof(LR), "strip copy", c, L.SO.n);
            const int p = c + lane < nso ? c + lane : nso - 1;
            lds_copy_word(so + c, lane, ring_f, rec_word(p, wlo) + (C::F32 ? (uint32_t)(H * F) : 0u));
        }
        if constexpr (C::F32) {
            const int nsh = 2 * t.npe * jm * H * F;
            float* const sh = &L.SOhi[0];
            for (int c = tid & ~63; c < nsh; c += nth) {
                AT_CHECK((int64_t)(c + 64) <= L.SOhi.n, "strip copy hi", c, L.SOhi.n);
                const int p = c + lane < nsh ? c + lane : nsh - 1;
                lds_copy_word(sh + c, lane, ring_f, rec_word(p, H * F));
            }
        }
    };
    // FP32 scalar kind: the halo of a PE side at every stage, extrapolated once per step
    // (hi part: level 0's; lo part: level 0's plus the weighted differences of the other
    // levels to it, in level order).  Levels below nreg are in registers (weights of
    // levels 1.. in wl), the others are loaded here.
    auto hq_put = [&](int side_idx, int ke, int jeff, int nreg, const LR (&rv)[JPR][nrec],
                      const float (&rvh)[JPR][nhi], const float (&wl)[JPR]) {
        float hi[nhi], lo[nrec];
#pragma unroll
        for (int r = 0; r < nhi; ++r) hi[r] = rvh[0][r];
#pragma unroll
        for (int r = 0; r < nrec; ++r) lo[r] = rv[0][r];
#pragma unroll
        for (int l = 1; l < JM; ++l) {
            if (l >= jeff) continue;
            LR v[nrec];
            float vh[nhi];
            float w;
            if (l < JPR && l < nreg) {
                const int lr = l < JPR ? l : 0;
#pragma unroll
                for (int r = 0; r < nrec; ++r) v[r] = rv[lr][r];
#pragma unroll
                for (int r = 0; r < nhi; ++r) vh[r] = rvh[lr][r];
                w = wl[lr];
            } else {
                ring_ld(side_idx, ke, l, v, vh);
                w = (float)WTAB.w[J][ke][l];
            }
#pragma unroll
            for (int r = 0; r < nrec; ++r) {
                const int hf = r % (H * F);       // record word r = (s H + h) F + f
                lo[r] += w * ((vh[hf] - hi[hf]) + (v[r] - rv[0][r]));
            }
        }
#pragma unroll
        for (int r = 0; r < nhi; ++r) L.SOhi[side_idx * H * F + r] = hi[r];
#pragma unroll
        for (int r = 0; r < nrec; ++r) L.SO[side_idx * L.SOREC + r] = lo[r];
    };
    // FP64 scalar kind: the halo of every stage, extrapolated once per step (the
    // weighted sum over the levels, level order, as the extrapolation of the other
    // kinds takes it).  Levels below nreg are in registers, the others are loaded here.
    auto hq_put64 = [&](int side_idx, int ke, int jeff, int nreg, const LR (&rv)[JPR][nrec]) {
        const int kw = ke == 0 ? 1 : J;          // the weights of delay 0 are one level's
        LR acc[nrec];
#pragma unroll
        for (int r = 0; r < nrec; ++r) acc[r] = LR(WTAB.w[kw][ke][0]) * rv[0][r];
#pragma unroll
        for (int l = 1; l < JM; ++l) {
            if (l >= jeff) continue;
            LR v[nrec];
            float vh[nhi];
            if (l < JPR && l < nreg) {
#pragma unroll
                for (int r = 0; r < nrec; ++r) v[r] = rv[l < JPR ? l : 0][r];
            } else {
                ring_ld(side_idx, ke, l, v, vh);
            }
            const LR w = LR(WTAB.w[kw][ke][l]);
#pragma unroll
            for (int r = 0; r < nrec; ++r) acc[r] += w * v[r];
        }
#pragma unroll
        for (int r = 0; r < nrec; ++r) L.SO[side_idx * L.SOREC + r] = acc[r];
    };
    rt.each([&](int tid, TS<C>& ts) {
        const int nraw = t.npts + 2 * SH;
        AT_CHECK(nraw <= nth * (PPT + 1), "raw range", nraw, nth * (PPT + 1));
        // loads of the raw range and of the first PE side's ring levels are all issued
        // before any of them is stored, so that their latencies overlap
        LR vh[RAW_DMA ? 1 : PPT + 1][F];
        float vl[RAW_DMA ? 1 : PPT + 1][F];
        // the range wraps round the periodic domain only in a problem's first and last tile
        const bool wraps = t.lo < SH || t.lo + t.npts + SH > N;
        const int Ni = (int)N, xs = (int)t.lo - SH;
        auto raw_x = [&](int r) -> int {
            int x = xs + r;
            if (wraps) {
                if (Ni >= SH) {
                    x = x < 0 ? x + Ni : x;
                    x = x >= Ni ? x - Ni : x;
                } else {
                    x = (int)wrapi(x, N);
                }
            }
            return x;
        };
        if constexpr (OWN_REG) {
            // own points into registers (inside [0, N): no wrap)
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int i = tid + k * nth;
                if (i >= t.npts) continue;
                const int64_t x = t.lo + i;
                ts.uh[k][0] = st.ld(x);
                ts.ul[k][0] = use_lo ? stlo.ld(x) : 0.f;
            }
            // the boundary windows of level n, straight into the window region: wave-sized
            // chunks of 64 consecutive window positions (the layout pads the region to a
            // multiple of 64); lanes past the last position copy its word
            if (first) {
                const int nwin = (t.npe + 1) * WL;
                const int lane = tid & 63;
                for (int c = tid & ~63; c < nwin; c += nth) {
                    const int wp = c + lane < nwin ? c + lane : nwin - 1;
                    const int b = wp / WL, w = wp - b * WL;
                    const int x = raw_x((int)(pe_offset(t.pe0 + b) - t.lo) + w);
                    AT_CHECK(x >= 0 && x < st.n, "window copy", x, st.n);
                    lds_copy_word(&L.wu[0][c], lane, st.p, (uint32_t)x);
                    if (use_lo) lds_copy_word(&L.wulo[0][c], lane, stlo.p, (uint32_t)x);
                    else L.wulo[0][c + lane] = 0.f;
                }
            }
        } else if constexpr (RAW_DMA) {
            // wave-sized chunks of 64 consecutive positions (the layout pads the range to
            // a multiple of 64); lanes past the end of the range copy its last word
            const int lane = tid & 63, wbase = tid & ~63;
#pragma unroll
            for (int k = 0; k <= PPT; ++k) {
                const int r0 = wbase + k * nth;
                if (r0 >= nraw) continue;
                const int r = r0 + lane < nraw ? r0 + lane : nraw - 1;
                const int x = raw_x(r);
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const int64_t gi = f * N + x;
                    AT_CHECK(gi >= 0 && gi < st.n, "raw copy", gi, st.n);
                    lds_copy_word(&L.rh[f][r0], lane, st.p, (uint32_t)gi);
                    if (use_lo) lds_copy_word(&L.rl[f][r0], lane, stlo.p, (uint32_t)gi);
                    else L.rl[f][r0 + lane] = 0.f;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k <= PPT; ++k) {
                const int r = tid + k * nth;
                if (r >= nraw) continue;
                const int x = raw_x(r);
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    vh[k][f] = st.ld(f * N + x);
                    vl[k][f] = use_lo ? stlo.ld(f * N + x) : 0.f;
                }
            }
        }
        const int si0 = first_item(tid, nth, 1);
        const bool has0 = si0 < 2 * t.npe;
        // scalar FD kind: the first PE side's levels in registers (extrapolated below);
        // the other kinds copy the strips straight into LDS
        constexpr int JR = C::KIND == K_ADR ? JPR : 1;
        LR rv[JR][nrec];
        float rvh[JR][nhi];
        float wl[JR];
        int jeff0 = 0, ke0 = 0;
        if (has0) {
            jeff0 = side_delays(si0, ke0);
            if constexpr (C::KIND == K_ADR) {
                if (!staged) {
#pragma unroll
                    for (int l = 0; l < JPF; ++l)
                        if (l < jeff0) ring_ld(si0, ke0, l, rv[l], rvh[l]);
                }
            }
            if constexpr (C::HILO) {
#pragma unroll
                for (int l = 1; l < JPF; ++l)
                    if (l < jeff0) wl[l] = (float)WTAB.w[J][ke0][l];
            }
        }
        for (int k = first_item(tid, nth, 3); k <= t.npe; k += nth)
            L.pelo[k] = (int)(pe_offset(t.pe0 + k) - t.lo);
        if (C::KIND != K_ADR && tid < 16 * JMAXW) {   // weights for delay k (J levels; k = 0 uses one level)
            const int k = tid / JMAXW, l = tid % JMAXW;
            L.wt[tid] = l < JM ? WTAB.w[k == 0 ? 1 : J][k][l] : 0.0;
        }
        if constexpr (!RAW_DMA) {
#pragma unroll
            for (int k = 0; k <= PPT; ++k) {
                const int r = tid + k * nth;
                if (r >= nraw) continue;
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    L.rh[f][r] = vh[k][f];
                    if constexpr (C::F32) L.rl[f][r] = vl[k][f];
                }
            }
        }
        if (staged) {
            // scalar FD kind, strips staged in LDS: delays of further PE sides, then the copies
            for (int side_idx = si0 + nth; side_idx < 2 * t.npe; side_idx += nth) {
                int ke;
                side_delays(side_idx, ke);
            }
            ring_copy(tid);
        } else if constexpr (C::HILO) {
            if (has0 && jeff0 > 0) hq_put(si0, ke0, jeff0, JPF, rv, rvh, wl);
            // further PE sides (tiles of more than nth / 2 PEs)
            for (int side_idx = si0 + nth; side_idx < 2 * t.npe; side_idx += nth) {
                int ke;
                const int jeff = side_delays(side_idx, ke);
                if (jeff == 0) continue;
                ring_ld(side_idx, ke, 0, rv[0], rvh[0]);
                hq_put(side_idx, ke, jeff, 1, rv, rvh, wl);
            }
        } else if constexpr (C::KIND == K_ADR) {
            if (has0 && jeff0 > 0) hq_put64(si0, ke0, jeff0, JPF, rv);
            // further PE sides (tiles of more than nth / 2 PEs)
            for (int side_idx = si0 + nth; side_idx < 2 * t.npe; side_idx += nth) {
                int ke;
                const int jeff = side_delays(side_idx, ke);
                if (jeff == 0) continue;
                ring_ld(side_idx, ke, 0, rv[0], rvh[0]);
                hq_put64(side_idx, ke, jeff, 1, rv);
            }
        } else {
            // delays (and log) of further PE sides (tiles of more than nth / 2 PEs)
            for (int side_idx = si0 + nth; side_idx < 2 * t.npe; side_idx += nth) {
                int ke;
                side_delays(side_idx, ke);
            }
            ring_copy(tid);
        }
        if (stage_io) {
            const GView<LR> kb{(LR*)P.kbuf, P.kbuf_len};
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int i = tid + k * nth;
                if (i >= t.npts) continue;
                const int64_t x = t.lo + i;
#pragma unroll
                for (int s = 0; s < S; ++s)
                    if (s < s0)
#pragma unroll
                        for (int f = 0; f < F; ++f) {
                            ts.K[s][k][f] = kb.ld(((int64_t)s * F + f) * N + x);
                            ts.acc[k][f] = s == 0 ? LR(TB::b(0)) * ts.K[s][k][f]
                                                  : ts.acc[k][f] + LR(TB::b(s)) * ts.K[s][k][f];
                        }
            }
        }
    });
    // the direct copies complete on the vector-memory counter: drained before the barrier
    if constexpr (RAW_DMA || C::KIND != K_ADR) rt.sync_mem();
    else rt.sync();

    // tile-local PE of own point i.  The PE owning global x = lo + i is ceil(z) - 1 with
    // z = (x + 1) P / N.  In FP32, z' = (i + 1) (P/N) + (lo P/N - pe0) is within 1e-4 of
    // z (z - pe0 <= npe <= 256, i < 4096), so floor(z' - 1e-3) is the PE or the one
    // before it; one comparison with the next PE offset decides.
    const float pn_f = (float)((double)Pp / (double)N);
    const float pe_c0 = (float)((double)t.lo * ((double)Pp / (double)N) - (double)t.pe0);
    auto pe_local = [&](int i) -> int {
        int pl = (int)floorf(fmaf((float)(i + 1), pn_f, pe_c0) - 1e-3f);
        pl = pl < 0 ? 0 : (pl >= t.npe ? t.npe - 1 : pl);
        if (L.pelo[pl + 1] <= i) ++pl;
        AT_CHECK(L.pelo[pl] <= i && i < L.pelo[pl + 1], "own point PE", i, pl);
        return pl;
    };

    // own stage state V(s) = u^n + dt sum_{i<s} a_si K_i of slot k, field f
    auto own_state = [&](const TS<C>& ts, int k, int f, auto sc, float& vlo) -> Q {
        constexpr int s = decltype(sc)::value;
        if constexpr (s == 0) {
            vlo = ts.ul[k][f];
            if constexpr (C::F32) return (Q)ts.uh[k][f] + (Q)ts.ul[k][f];
            else return (Q)ts.uh[k][f];
        } else {
            // sum_{i<s} a_si K_i, i ascending; zero coefficients are skipped at compile
            // time so that a K_i no later stage needs is not kept in registers
            LR acc = LR(0);
            bool have = false;
            static_for<0, s>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if constexpr (TB::a(s, i) != 0.0) {
                    acc = have ? acc + LR(TB::a(s, i)) * ts.K[i][k][f] : LR(TB::a(s, i)) * ts.K[i][k][f];
                    have = true;
                }
            });
            if constexpr (C::F32) {
                const float lo = ts.ul[k][f] + PP.dtf * acc;
                vlo = lo;
                return (Q)ts.uh[k][f] + (Q)lo;
            } else {
                vlo = 0.f;
                return (Q)(ts.uh[k][f] + dt * acc);
            }
        }
    };
    // own slot k of thread tid: whether it holds a point, and the point's ext position
    // (the FP32 scalar kind keeps e - H, known non-negative, so that its LDS neighbours sit
    // at non-negative offsets)
    auto pt_ok = [&](const TS<C>& ts, int tid, int k) -> bool {
        if constexpr (C::HILO) return tid + k * nth < t.npts;
        else return ts.e[k] >= 0;
    };
    auto pt_e = [&](const TS<C>& ts, int k) -> int {
        if constexpr (C::HILO) return (int)ts.eb[k] + H;
        else return ts.e[k];
    };
    // quantities of V(s) at own slot k, into the main region of stage parity s & 1
    auto own_quant = [&](TS<C>& ts, int k, auto sc) {
        constexpr int s = decltype(sc)::value;
        const QV<C>& M = L.main[s & 1];
        const int e = pt_e(ts, k);
        Q q[F];
        float vlo[F];
#pragma unroll
        for (int f = 0; f < F; ++f) q[f] = own_state(ts, k, f, sc, vlo[f]);
        if constexpr (C::HILO) {
            if (s == s0) M.g[0][e] = ts.uh[k][0];   // hi: fixed within the step, both parities
            M.glo[2 * (int64_t)e] = vlo[0];
        } else if constexpr (C::KIND == K_REUL) {
            put_quant<C>(M, PP, e, q, &ts.src[k]);  // and the source of the stage's right-hand side
        } else {
            put_quant<C>(M, PP, e, q);
        }
    };
    // ext position of halo point h on the given side of tile PE k
    auto halo_e = [&](int k, int side, int h) -> int {
        const int ebase = L.pelo[k] + 2 * H * k;
        return side == 0 ? ebase + h : ebase + H + (L.pelo[k + 1] - L.pelo[k]) + h;
    };
    // halo point h of a PE side at stage s: the differentiated quantities of the delayed
    // strips (levels n - ke - l), extrapolated in time to level n with the Lagrange
    // weights of the delay (per-stage entry point with delay 0: level n's own strip)
    auto halo_from_so = [&](int side_idx, int h, auto sc) {
        constexpr int s = decltype(sc)::value;
        const QV<C>& M = L.main[s & 1];
        const int e = halo_e(side_idx >> 1, side_idx & 1, h);
        const int sob = side_idx * L.SOREC;
        if (C::KIND == K_ADR && staged) {
            // the staged levels, extrapolated here as the load phase does it with the
            // strips in registers (same operations, same order)
            const int ke = L.keff[side_idx];
            const int jeff = ke == 0 ? 1 : J;
            const int hb = side_idx * L.jmax * H * F;       // FP32 hi words of level 0
            const int wofs = (s * H + h) * F;               // the stage's word in a level
            if constexpr (C::HILO) {
                const float hi0 = L.SOhi[hb + h * F];
                const float lo0 = L.SO[sob + wofs];
                float lo = lo0;
#pragma unroll
                for (int l = 1; l < JM; ++l) {
                    if (l >= jeff) continue;
                    const float w = (float)WTAB.w[J][ke][l];
                    lo += w * ((L.SOhi[hb + l * H * F + h * F] - hi0) + (L.SO[sob + l * S * H * F + wofs] - lo0));
                }
                if (s == s0) M.g[0][e] = hi0;
                M.glo[2 * (int64_t)e] = lo;
            } else {
                const int kw = ke == 0 ? 1 : J;
                LR acc = LR(WTAB.w[kw][ke][0]) * L.SO[sob + wofs];
#pragma unroll
                for (int l = 1; l < JM; ++l) {
                    if (l >= jeff) continue;
                    acc += LR(WTAB.w[kw][ke][l]) * L.SO[sob + l * S * H * F + wofs];
                }
                M.g[0][e] = acc;
            }
        } else if constexpr (C::HILO) {
            // extrapolated in the load phase
            if (s == s0) M.g[0][e] = L.SOhi[side_idx * H * F + h * F];
            M.glo[2 * (int64_t)e] = L.SO[sob + (s * H + h) * F];
        } else if constexpr (C::KIND == K_ADR) {
            M.g[0][e] = L.SO[sob + (s * H + h) * F];   // extrapolated in the load phase
        } else {
            const int ke = L.keff[side_idx];
            const int jeff = ke == 0 ? 1 : J;
            double w[JM];
#pragma unroll
            for (int l = 0; l < JM; ++l) w[l] = L.wt[ke * JMAXW + l];
            const int sohb = side_idx * L.jmax;
            Q gl[NQ], g0[NQ], acc[NQ];
            Q lam0 = Q(0), laml = Q(0);
#pragma unroll
            for (int l = 0; l < JM; ++l) {
                if (l >= jeff) continue;
                Q q[F];
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    const LR v = L.SO[sob + ((l * S + s) * H + h) * F + f];
                    if constexpr (C::F32) q[f] = (Q)L.SOhi[((sohb + l) * H + h) * F + f] + (Q)v;
                    else q[f] = (Q)v;
                }
                quant_values<C>(PP, q, gl, laml);
                if (l == 0) {
                    lam0 = laml;
#pragma unroll
                    for (int j = 0; j < NQ; ++j) {
                        g0[j] = gl[j];
                        acc[j] = C::F32 ? gl[j] : Q(w[0]) * gl[j];
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < NQ; ++j) {
                        if constexpr (C::F32) acc[j] += Q(w[l]) * (gl[j] - g0[j]);
                        else acc[j] += Q(w[l]) * gl[j];
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < NQ; ++j) M.g[j][e] = (LR)acc[j];
            if constexpr (C::WENO) M.lam[e] = (LR)lam0;
        }
    };

    // ---- P2: own points and boundary windows from the staged raw range --------------
    rt.each([&](int tid, TS<C>& ts) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int i = tid + k * nth;
            if constexpr (!C::HILO) ts.e[k] = -1;
            if constexpr (C::KIND == K_REUL) ts.src[k] = LR(0);
            // every per-point register gets a value on every path, so that none of them is
            // live across the tile loop (a slot without a point is never read)
            if constexpr (C::HILO) {
                ts.eb[k] = 0;
                ts.khi[k] = 0.f;
                // (the per-stage entry point has loaded sum_{s<s0} b_s K_s already)
                if (!stage_io) ts.acc[k][0] = 0.f;
            }
            if constexpr (WENO_DPP) ts.eb[k] = 0;
            if (i >= t.npts) continue;
            const int lo = pe_local(i);
            if constexpr (C::HILO) ts.eb[k] = (uint32_t)(i + 2 * H * lo) & 0xFFFFu;
            else ts.e[k] = i + 2 * H * lo + H;
            if constexpr (WENO_DPP && C::WENO) {
                // lanes -2..+3 hold points of the same PE (build option)
                const int lane = tid & 63;
                ts.eb[k] = lane >= 2 && lane <= 60 && i >= 2 && i + 3 < t.npts && pe_local(i - 2) == lo &&
                           pe_local(i + 3) == lo;
            }
            if constexpr (!OWN_REG) {
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    ts.uh[k][f] = L.rh[f][i + SH];
                    ts.ul[k][f] = C::F32 ? L.rl[f][i + SH] : 0.f;
                }
            }
        }
        if (OWN_REG && first) {
            // the windows are in place: stage-0 records of level n of the halo positions
            for (int idx = first_item(tid, nth, 0); idx < (t.npe + 1) * 2 * H; idx += nth) {
                const int b = idx / (2 * H), w = (S - 1) * H + (idx - b * 2 * H);
                const int wp = b * WL + w;
                strip_out(b, w, 0, 0, L.wulo[0][wp], L.wu[0][wp]);
            }
        }
        if (!OWN_REG && first) {
            for (int idx = first_item(tid, nth, 0); idx < (t.npe + 1) * WL; idx += nth) {
                const int b = idx / WL, w = idx - b * WL;
                const int r = L.pelo[b] + w;       // raw index of window position w
                const int wp = b * WL + w;
                Q q[F];
                LR hv[F];
                float lv[F];
#pragma unroll
                for (int f = 0; f < F; ++f) {
                    hv[f] = L.rh[f][r];
                    lv[f] = C::F32 ? L.rl[f][r] : 0.f;
                    L.wu[f][wp] = hv[f];
                    if constexpr (C::F32) {
                        L.wulo[f][wp] = lv[f];
                        L.wq[0][f][wp] = lv[f];
                        q[f] = (Q)hv[f] + (Q)lv[f];
                    } else {
                        L.wq[0][f][wp] = hv[f];
                        q[f] = (Q)hv[f];
                    }
                    strip_out(b, w, 0, f, C::F32 ? (LR)lv[f] : hv[f], (float)hv[f]);
                }
                // FP32 scalar kind: the window's quantities are the state just written
                if constexpr (!C::HILO) put_quant<C>(L.win[0], PP, wp, q);
            }
        }
    });
    // with own points in registers and the windows in place, the first stage's
    // quantities below read nothing this phase wrote
    if constexpr (!OWN_REG) rt.sync();

    // ---- A0: quantities of the first stage at own and halo points --------------------
    static_for<0, S>([&](auto sc) {
        if (decltype(sc)::value != s0) return;
        rt.each([&](int tid, TS<C>& ts) {
#pragma unroll
            for (int k = 0; k < PPT; ++k)
                if (pt_ok(ts, tid, k)) own_quant(ts, k, sc);
            for (int idx = first_item(tid, nth, 2); idx < 2 * t.npe * H; idx += nth) {
                const int side_idx = idx / H, h = idx - side_idx * H;
                if (first && L.keff[side_idx] == 0) {
                    // synchronous stage 0 of level n: the window's value at the halo point
                    const int k = side_idx >> 1, side = side_idx & 1;
                    const int wp = (k + side) * WL + (S - 1) * H + side * H + h;
                    const int e = halo_e(k, side, h);
                    const QV<C>& M = L.main[0];
                    const QV<C>& W0 = C::HILO ? L.win0 : L.win[0];
#pragma unroll
                    for (int j = 0; j < NQ; ++j) M.g[j][e] = W0.g[j][wp];
                    if constexpr (C::HILO) M.glo[2 * (int64_t)e] = W0.glo[wp];
                    if constexpr (C::WENO) M.lam[e] = W0.lam[wp];
                } else {
                    halo_from_so(side_idx, h, sc);
                }
            }
        });
    });
    rt.sync();

    // ---- the stages: one phase each (two for WENO) ----------------------------------
    //   stage s reads the main region of parity s & 1 and writes the quantities of
    //   stage s + 1 (own points, halo points, windows) into parity (s + 1) & 1
    static_for<0, S>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int sn = s + 1 < S ? s + 1 : s;                 // next stage (if any)
        using SN = std::integral_constant<int, sn>;
        const bool own_active = s >= s0 && s <= s1;
        const bool next_active = s + 1 < S && own_active && s + 1 <= s1;
        const bool win_active = first && s + 1 < S;
        if (!own_active && !win_active) return;
        const QV<C>& Mc = L.main[s & 1];
        const QV<C>& Mn = L.main[sn & 1];
        const QV<C>& Wc = (C::HILO && s == 0) ? L.win0 : L.win[s & 1];   // stage 0: u^n
        const QV<C>& Wn = L.win[(s + 1) & 1];

        // B1 (WENO): interface fluxes, the phase compiled once per form (reconstruction or
        // interpolation) and chosen by a uniform branch around it
        if constexpr (C::WENO) {
            auto fluxes = [&](auto form) {
                constexpr bool INTERP = decltype(form)::value;
                rt.each([&](int tid, TS<C>& ts) {
                    if (own_active) {
#pragma unroll
                        for (int k = 0; k < PPT; ++k) {
                            const int e = ts.e[k];
                            if (k > 0) sched_fence();
                            // right interface of the point
                            if (e >= 0)
                                iface_flux_form<C, WENO_DPP && C::F32, INTERP>(Mc, PP, e, ts.eb[k] != 0);
                        }
                        // left interface of each PE's first point (its left neighbour is a
                        // halo slot), as a short work list of its own
                        sched_fence();
                        for (int b = first_item(tid, nth, 2 * s + 2); b < t.npe; b += nth)
                            iface_flux_form<C, false, INTERP>(Mc, PP, L.pelo[b] + 2 * H * b + H - 1, false);
                    }
                    if (win_active) {
                        const int rlo = (s + 1) * H, rhi = WL - (s + 1) * H;
                        const int ni = rhi - rlo + 1;                 // interfaces rlo-1 .. rhi-1
                        for (int idx = first_item(tid, nth, 2 * s + 1); idx < (t.npe + 1) * ni; idx += nth) {
                            const int b = idx / ni, j = rlo - 1 + (idx - b * ni);
                            iface_flux_form<C, false, INTERP>(Wc, PP, b * WL + j, false);
                        }
                    }
                });
            };
            if (PP.interp) fluxes(std::true_type{});
            else fluxes(std::false_type{});
            rt.sync();
        }

        // B2: K_s at own points and the quantities of stage s+1; R_s and the synchronous
        // stage s+1 on the windows
        rt.each([&](int tid, TS<C>& ts) {
            if (own_active) {
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    if (k > 0 && (C::WENO || (C::HILO && k % 2 == 0))) sched_fence();
                    if (!pt_ok(ts, tid, k)) continue;
                    const int e = pt_e(ts, k);
                    Q q[F];
                    float vlo = 0.f;
                    if constexpr (!C::HILO) {
#pragma unroll
                        for (int f = 0; f < F; ++f) q[f] = own_state(ts, k, f, sc, vlo);
                    }
                    LR K[F];
                    if constexpr (C::HILO) {
                        // the hi parts' share once per step (stage s0 of the launch)
                        const float hc = ts.uh[k][0];
                        if (s == s0) {
                            float kh = 0.f;
#pragma unroll
                            for (int o = H; o >= 1; --o) {
                                kh = fmaf(PP.lmf[o - 1], Mc.g[0][e - o] - hc, kh);
                                kh = fmaf(PP.lpf[o - 1], Mc.g[0][e + o] - hc, kh);
                            }
                            ts.khi[k] = kh;
                        }
                        float lc;      // the stage's lo part of the point, as own_quant wrote it
                        const float lsum = hilo_lo_sum<C>(L.main[0].glo, ts.eb[k], s & 1, PP, lc);
                        const float u = hc + lc;
                        float kk = fmaf(-PP.c0f, lc, ts.khi[k] + lsum);
                        K[0] = fmaf(PP.rlf * u, 1.f - u, kk);
                    } else {
                        const int64_t xg = t.lo + tid + k * nth;
                        if constexpr (C::KIND == K_RNS) {
                            if (P.bc == 1 && (xg < H || xg >= N - H)) {
                                double qd[F];
#pragma unroll
                                for (int f = 0; f < F; ++f) qd[f] = (double)q[f];
                                rhs_end_rns<C>(Mc, PP, e, xg, N, qd, K);
                            } else {
                                rhs_at<C>(Mc, PP, e, q, K);
                            }
                        } else if constexpr (C::KIND == K_REUL) {
                            rhs_at<C>(Mc, PP, e, q, K, &ts.src[k]);
                        } else {
                            rhs_at<C>(Mc, PP, e, q, K);
                        }
                    }
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        ts.K[s][k][f] = K[f];
                        ts.acc[k][f] = s == 0 ? LR(TB::b(0)) * K[f] : ts.acc[k][f] + LR(TB::b(s)) * K[f];
                    }
                    if (stage_io && s == s1 && s1 < S - 1) {   // per-stage entry point: K_s out
                        const GView<LR> kb{(LR*)P.kbuf, P.kbuf_len};
                        const int64_t x = t.lo + tid + k * nth;
#pragma unroll
                        for (int f = 0; f < F; ++f) kb.st(((int64_t)s * F + f) * N + x, K[f]);
                    }
                    if constexpr (s + 1 < S)
                        if (next_active) own_quant(ts, k, SN{});
                }
            }
            if constexpr (s + 1 < S) {
                if (next_active) {
                    for (int idx = first_item(tid, nth, s + 3); idx < 2 * t.npe * H; idx += nth) {
                        const int side_idx = idx / H, h = idx - side_idx * H;
                        if (!(first && L.keff[side_idx] == 0)) halo_from_so(side_idx, h, SN{});
                    }
                }
            }
            if (win_active) {
                const int rlo = (s + 1) * H, rhi = WL - (s + 1) * H;
                const int nr = rhi - rlo;
                for (int idx = first_item(tid, nth, 2 * s); idx < (t.npe + 1) * nr; idx += nth) {
                    const int b = idx / nr, w = rlo + (idx - b * nr);
                    const int wp = b * WL + w;
                    Q q[F];
                    float whi = 0.f, wlo = 0.f;
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        if constexpr (C::F32) {
                            whi = L.wu[f][wp];
                            wlo = (C::HILO && s == 0) ? L.wulo[f][wp] : L.wq[s & 1][f][wp];
                            q[f] = (Q)whi + (Q)wlo;
                        } else {
                            q[f] = (Q)L.wq[s & 1][f][wp];
                        }
                    }
                    LR K[F];
                    if constexpr (C::HILO) K[0] = rhs_adr_hilo<C>(Wc, PP, wp, whi, wlo);
                    else rhs_at<C>(Wc, PP, wp, q, K);
                    Q qn[F];
                    LR hv[F];
                    float lvn[F];
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        if constexpr (rk_keeps_stage_rhs<S>()) L.wR[s][f][wp] = K[f];
                        // sum_{i <= s} a_{s+1,i} R_i, ascending i, zero coefficients skipped
                        LR acc = LR(0);
                        bool have = false;
                        static_for<0, s + 1>([&](auto ic) {
                            constexpr int i = decltype(ic)::value;
                            if constexpr (TB::a(s + 1, i) != 0.0) {
                                const LR r = i == s ? K[f] : L.wR[i][f][wp];
                                acc = have ? acc + LR(TB::a(s + 1, i)) * r : LR(TB::a(s + 1, i)) * r;
                                have = true;
                            }
                        });
                        hv[f] = L.wu[f][wp];
                        if constexpr (C::F32) {
                            const float lo = L.wulo[f][wp] + PP.dtf * acc;
                            lvn[f] = lo;
                            L.wq[(s + 1) & 1][f][wp] = lo;
                            qn[f] = (Q)hv[f] + (Q)lo;
                        } else {
                            const LR v = hv[f] + dt * acc;
                            lvn[f] = 0.f;
                            L.wq[(s + 1) & 1][f][wp] = v;
                            qn[f] = (Q)v;
                        }
                    }
                    // FP32 scalar kind: the window's quantities are its state (hi in wu, lo in
                    // the stage parity's wq, written above), nothing more to write
                    if constexpr (!C::HILO) put_quant<C>(Wn, PP, wp, qn);
                    // a halo point (left of PE b or right of PE b - 1): its ring record of stage
                    // s + 1 and, for a PE side of delay 0, its stage s + 1 quantities
                    const int h2 = w - (S - 1) * H;
                    if ((unsigned)h2 < (unsigned)(2 * H)) {
                        const int side = h2 < H ? 0 : 1, kpe = b - side, h = h2 - side * H;
                        if ((unsigned)kpe < (unsigned)t.npe) {
#pragma unroll
                            for (int f = 0; f < F; ++f)
                                rec_store(kpe, side, s + 1, h, f, C::F32 ? (LR)lvn[f] : (LR)qn[f], 0.f);
                            if (next_active && L.keff[2 * kpe + side] == 0) {
                                const int e = halo_e(kpe, side, h);
                                if constexpr (C::HILO) Mn.glo[2 * (int64_t)e] = lvn[0];
                                else put_quant<C>(Mn, PP, e, qn);
                            }
                        }
                    }
                }
            }
        });
        if (s + 1 < S && (next_active || (first && s + 2 < S))) rt.sync();
    });

    // ---- P5: the update (or the stage output of the per-stage entry point) ----------
    rt.each([&](int tid, TS<C>& ts) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!pt_ok(ts, tid, k)) continue;
            const int64_t x = t.lo + tid + k * nth;
            if (s1 < S - 1) continue;              // per-stage entry point: K_s1 already out
            const GView<LR> dst = st_view<C>(P, nxt);
            const GView<float> dlo = lo_view(P, nxt, C::F32);
#pragma unroll
            for (int f = 0; f < F; ++f) {
                const LR acc = ts.acc[k][f];       // sum_s b_s K_s, s ascending
                if constexpr (C::F32) {
                    // compensated update: (hi, lo) + dt*acc, TwoSum of hi and (lo + dt*acc)
                    const float hi = ts.uh[k][f];
                    const float tt = ts.ul[k][f] + PP.dtf * acc;
                    const float sum = hi + tt;
                    const float bb = sum - hi;
                    const float err = (hi - (sum - bb)) + (tt - bb);
                    dst.st(f * N + x, sum);
                    if (P.keep_lo) dlo.st(f * N + x, err);
                } else {
                    dst.st(f * N + x, (LR)(ts.uh[k][f] + dt * acc));
                }
            }
        }
    });
}

}  // namespace atk
