// at_emu.cpp -- CPU emulation of libat's tile kernels (test infrastructure).
//
// Runs the exact tile code of the gfx950 kernels (at_tile.hpp) on the host,
// one "thread" after another inside each barrier-delimited phase, with every
// LDS and global access bounds-checked and LDS / per-thread registers poisoned
// with NaN before use.  It shares the planner and the workspace layout with
// the HIP library, so index or layout mistakes show up here before a kernel
// ever runs on a GPU.  It is not a fallback: the product library has no CPU
// path and never loads this file.
#define AT_EMU 1
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "at_plan.hpp"
#include "at_variants.hpp"

namespace {
struct EmuFail : std::runtime_error {
    using std::runtime_error::runtime_error;
};
}  // namespace

void at_emu_fail(const char* what, const char* file, int line, long long i, long long n) {
    char buf[512];
    snprintf(buf, sizeof(buf), "bounds check '%s' failed at %s:%d (index %lld, size %lld)", what,
             file, line, i, n);
    throw EmuFail(buf);
}

namespace atk {

template <class C>
struct CpuRT {
    std::vector<TS<C>> ts;
    CpuRT() : ts(BLOCK) {
        for (auto& t : ts) std::memset(&t, 0xff, sizeof(t));   // NaN / -1 poison
    }
    int nthreads() const { return BLOCK; }
    template <class Fn>
    void each(Fn&& f) {
        for (int t = 0; t < BLOCK; ++t) f(t, ts[t]);
    }
    void sync() {}
    void sync_mem() {}
};

struct EmuCtx {
    Plan plan;
    std::vector<unsigned char> ws;
    unsigned char* base = nullptr;
    int64_t step = 0;
    int stage = 0;                       // next stage (0-based) of at_rk_stage
    std::vector<int64_t> ov_step0, ov_n;
    std::string err;
};

static void sync_probs(EmuCtx& c) {
    ProbDev* pd = (ProbDev*)(c.base + c.plan.off_probs);
    for (size_t b = 0; b < c.plan.desc.size(); ++b)
        fill_probdev(c.plan, (int)b, c.base, pd[b], c.ov_step0[b], c.ov_n[b]);
}

template <class C>
static void run_group(EmuCtx& c, const Group& g, int s_begin, int s_end, int flags) {
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.tiles = c.plan.tiles_bt.data() + g.t0;
    a.probs = (const ProbDev*)(c.base + c.plan.off_probs);
    a.step_ptr = nullptr;
    a.step_off = c.step;
    a.ntiles = g.ntiles;
    a.npts_max = g.npts_max;
    a.npe_max = g.npe_max;
    a.jmax = g.jmax;
    a.s_begin = s_begin;
    a.s_end = s_end;
    a.flags = flags;
    a.lds_bytes = (int32_t)g.lds_bytes;
    std::vector<unsigned char> lds((size_t)g.lds_bytes + 16);
    for (int ti = 0; ti < g.ntiles; ++ti) {
        std::memset(lds.data(), 0xff, lds.size());
        CpuRT<C> rt;
        const Tile& t = a.tiles[ti];
        const bool whole = s_begin == 0 && s_end == C::S - 1 && !(flags & KF_STAGE_IO);
        const bool staged = C::KIND == K_ADR && (flags & KF_HALO_LDS);
        if (whole)
            staged ? tile_step<C, true, true>(rt, a, t, a.probs[t.prob], c.step, lds.data())
                   : tile_step<C, true, false>(rt, a, t, a.probs[t.prob], c.step, lds.data());
        else
            staged ? tile_step<C, false, true>(rt, a, t, a.probs[t.prob], c.step, lds.data())
                   : tile_step<C, false, false>(rt, a, t, a.probs[t.prob], c.step, lds.data());
    }
}

// s_end < 0: every group runs all of its own stages (fused step)
static int run_all(EmuCtx& c, int s_begin, int s_end, int flags) {
    for (const Group& g : c.plan.groups) {
        const int se = s_end < 0 ? g.key.S - 1 : s_end;
        bool done = false;
#define AT_EMU_CASE(K, H_, S_, F32_, PPT_)                                                \
        if (!done && g.key.kind == (K) && g.key.H == (H_) && g.key.S == (S_) &&          \
            g.key.f32 == ((F32_) != 0) && g.key.ppt == (PPT_)) {                        \
            run_group<AT_CFG(K, H_, S_, F32_, PPT_)>(c, g, s_begin, se, flags);         \
            done = true;                                                                 \
        }
        AT_VARIANTS(AT_EMU_CASE)
#undef AT_EMU_CASE
        if (!done) {
            c.err = "variant not compiled";
            return AT_EUNSUPPORTED;
        }
    }
    return AT_OK;
}

}  // namespace atk

using namespace atk;

extern "C" {

int emu_init(const at_problem_desc* probs, int n, const at_run_opts* opts, void** out) {
    EmuCtx* c = new EmuCtx();
    int rc = make_plan(probs, n, opts, c->plan, c->err);
    if (rc) {
        *out = c;
        return rc;
    }
    c->ws.assign(c->plan.total + 256, 0);
    c->base = (unsigned char*)(((uintptr_t)c->ws.data() + 255) & ~uintptr_t(255));
    // poison the state and ring so that reads of never-written data give NaN
    std::memset(c->base, 0xff, c->plan.total);
    std::memcpy(c->base + c->plan.off_peoff, c->plan.peoff.data(), sizeof(int32_t) * c->plan.peoff.size());
    c->ov_step0.assign(n, 0);
    c->ov_n.assign(n, 0);
    sync_probs(*c);
    *out = c;
    return AT_OK;
}

const char* emu_error(void* ctx) { return ((EmuCtx*)ctx)->err.c_str(); }

void emu_free(void* ctx) { delete (EmuCtx*)ctx; }

int emu_set_state(void* ctx, int prob, const double* q) {
    EmuCtx& c = *(EmuCtx*)ctx;
    if (prob < 0 || prob >= (int)c.plan.desc.size()) return AT_EINVAL;
    c.step = 0;
    c.stage = 0;
    const ProbInfo& pi = c.plan.info[prob];
    const int prec = c.plan.desc[prob].precision;
    if (prec == AT_FP64) {
        std::memcpy(c.base + pi.off_hi[0], q, 8 * (size_t)pi.st_elems);
    } else {
        float* hi = (float*)(c.base + pi.off_hi[0]);
        float* lo = (float*)(c.base + pi.off_lo[0]);
        for (int64_t i = 0; i < pi.st_elems; ++i) {
            hi[i] = (float)q[i];
            if (prec == AT_FP32C) lo[i] = (float)(q[i] - (double)hi[i]);
        }
    }
    return AT_OK;
}

int emu_get_state(void* ctx, int prob, double* out) {
    EmuCtx& c = *(EmuCtx*)ctx;
    if (prob < 0 || prob >= (int)c.plan.desc.size()) return AT_EINVAL;
    const ProbInfo& pi = c.plan.info[prob];
    const int w = (int)(c.step & 1);
    const int prec = c.plan.desc[prob].precision;
    if (prec == AT_FP64) {
        std::memcpy(out, c.base + pi.off_hi[w], 8 * (size_t)pi.st_elems);
    } else {
        const float* hi = (const float*)(c.base + pi.off_hi[w]);
        const float* lo = (const float*)(c.base + pi.off_lo[w]);
        for (int64_t i = 0; i < pi.st_elems; ++i)
            out[i] = (double)hi[i] + (prec == AT_FP32C ? (double)lo[i] : 0.0);
    }
    return AT_OK;
}

int emu_step(void* ctx, int n_steps) {
    EmuCtx& c = *(EmuCtx*)ctx;
    if (c.stage != 0) return AT_ESTATE;
    try {
        for (int i = 0; i < n_steps; ++i) {
            const int flags = (c.plan.opts.log_steps ? KF_LOG : 0) | (c.plan.opts.halo_lds ? KF_HALO_LDS : 0);
            const int rc = run_all(c, 0, -1, flags);
            if (rc) return rc;
            c.step += 1;
        }
    } catch (const std::exception& e) {
        c.err = e.what();
        return AT_EINVAL;
    }
    return AT_OK;
}

int emu_rk_stage(void* ctx, int stage) {
    EmuCtx& c = *(EmuCtx*)ctx;
    const int S = c.plan.info[0].S;
    for (const ProbInfo& pi : c.plan.info)
        if (pi.S != S) {
            c.err = "per-stage stepping needs one RK scheme for all problems";
            return AT_EUNSUPPORTED;
        }
    if (!c.plan.opts.stage_api) return AT_ESTATE;
    if (stage != c.stage + 1 || stage < 1 || stage > S) return AT_ESTATE;
    try {
        int flags = KF_STAGE_IO | (c.plan.opts.log_steps ? KF_LOG : 0) | (c.plan.opts.halo_lds ? KF_HALO_LDS : 0);
        int rc = run_all(c, stage - 1, stage - 1, flags);
        if (rc) return rc;
    } catch (const std::exception& e) {
        c.err = e.what();
        return AT_EINVAL;
    }
    c.stage = stage;
    if (stage == S) {
        c.stage = 0;
        c.step += 1;
    }
    return AT_OK;
}

int emu_get_delays(void* ctx, int prob, int64_t step0, int n_steps, uint8_t* drawn, uint8_t* eff) {
    EmuCtx& c = *(EmuCtx*)ctx;
    const int64_t cap = c.plan.opts.log_steps;
    if (prob < 0 || prob >= (int)c.plan.desc.size() || cap == 0) return AT_EINVAL;
    if (step0 < 0 || step0 + n_steps > c.step || step0 < c.step - cap) return AT_ERANGE;
    const ProbInfo& pi = c.plan.info[prob];
    const int64_t P = c.plan.desc[prob].p;
    const uint8_t* ld = c.base + pi.off_log_d;
    const uint8_t* le = c.base + pi.off_log_e;
    for (int i = 0; i < n_steps; ++i) {
        const int64_t slot = (step0 + i) % cap;
        std::memcpy(drawn + (int64_t)i * P * 2, ld + slot * P * 2, (size_t)P * 2);
        std::memcpy(eff + (int64_t)i * P * 2, le + slot * P * 2, (size_t)P * 2);
    }
    return AT_OK;
}

int emu_set_override(void* ctx, int prob, const uint8_t* sched, int64_t step0, int n_steps) {
    EmuCtx& c = *(EmuCtx*)ctx;
    if (prob < 0 || prob >= (int)c.plan.desc.size()) return AT_EINVAL;
    if (n_steps < 0 || n_steps > c.plan.opts.override_steps) return AT_EINVAL;
    const int64_t P = c.plan.desc[prob].p;
    for (int64_t i = 0; i < (int64_t)n_steps * P * 2; ++i)
        if (sched[i] > c.plan.desc[prob].kmax) return AT_ESTALE;
    if (n_steps) std::memcpy(c.base + c.plan.info[prob].off_ov, sched, (size_t)n_steps * P * 2);
    c.ov_step0[prob] = step0;
    c.ov_n[prob] = n_steps;
    sync_probs(c);
    return AT_OK;
}

int64_t emu_query(void* ctx, int key) {
    EmuCtx& c = *(EmuCtx*)ctx;
    switch (key) {
    case AT_Q_STEP: return c.step;
    case AT_Q_NUM_TILES: return (int64_t)c.plan.tiles_bt.size();
    case AT_Q_NUM_GROUPS: return (int64_t)c.plan.groups.size();
    case AT_Q_TOTAL_POINTS: return c.plan.total_points;
    case AT_Q_STATE_BYTES: return c.plan.state_bytes_per_step;
    case AT_Q_STRIP_BYTES: return c.plan.strip_bytes_per_step;
    case AT_Q_NUM_PES: return c.plan.total_pes;
    case AT_Q_LDS_BYTES: {
        int64_t m = 0;
        for (const Group& g : c.plan.groups) m = g.lds_bytes > m ? g.lds_bytes : m;
        return m;
    }
    }
    return -1;
}

}  // extern "C"
