// at_plan.cpp -- validation, tiling and workspace layout (see at_plan.hpp).
#include "at_plan.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>

#include "at_variants.hpp"

namespace atk {

namespace {
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

std::string fmt(const char* f, long long a = 0, long long b = 0, long long c = 0) {
    char buf[256];
    snprintf(buf, sizeof(buf), f, a, b, c);
    return buf;
}
}  // namespace

bool variant_sizes(const VariantKey& v, int npts_max, int npe_max, int jmax, int64_t* lds_bytes,
                   int64_t* rec_bytes, bool halo_lds) {
#define AT_SIZE_CASE(K, H_, S_, F32_, PPT_)                                        \
    if (v.kind == (K) && v.H == (H_) && v.S == (S_) && v.f32 == ((F32_) != 0) &&   \
        v.ppt == (PPT_)) {                                                         \
        using C = AT_CFG(K, H_, S_, F32_, PPT_);                                   \
        Layout<C> lo;                                                              \
        lo.init(npts_max, npe_max, jmax, halo_lds);                                \
        *lds_bytes = lo.total;                                                     \
        *rec_bytes = record_bytes<C>();                                            \
        return true;                                                               \
    }
    AT_VARIANTS(AT_SIZE_CASE)
#undef AT_SIZE_CASE
    return false;
}

int rk_tableau(int rk, int* S, double a[MAXS][MAXS], double b[MAXS]) {
    for (int i = 0; i < MAXS; ++i) {
        b[i] = 0.0;
        for (int j = 0; j < MAXS; ++j) a[i][j] = 0.0;
    }
    switch (rk) {
    case AT_FE: *S = 1; b[0] = 1.0; return 0;
    case AT_RK2: *S = 2; a[1][0] = 1.0; b[0] = 0.5; b[1] = 0.5; return 0;
    case AT_SSPRK3:
        *S = 3; a[1][0] = 1.0; a[2][0] = 0.25; a[2][1] = 0.25;
        b[0] = 1.0 / 6.0; b[1] = 1.0 / 6.0; b[2] = 2.0 / 3.0; return 0;
    case AT_RK4:
        *S = 4; a[1][0] = 0.5; a[2][1] = 0.5; a[3][2] = 1.0;
        b[0] = 1.0 / 6.0; b[1] = 1.0 / 3.0; b[2] = 1.0 / 3.0; b[3] = 1.0 / 6.0; return 0;
    }
    return -1;
}

int fields_of(int pde) {
    switch (pde) {
    case AT_PDE_ADV_DIFF: case AT_PDE_ADR_LOGISTIC: case AT_PDE_BURGERS: return 1;
    case AT_PDE_EULER: return 3;
    case AT_PDE_REACTIVE_EULER: case AT_PDE_REACTIVE_NS: return 4;
    }
    return -1;
}

int halo_of(int scheme) {
    switch (scheme) {
    case AT_FD2: return 1;
    case AT_FD4: return 2;
    case AT_FD8: return 4;
    case AT_WENO5: case AT_WENO5I: return 3;
    }
    return -1;
}

// Time levels of the AT extrapolation: 3 for the 4th- and 8th-order central
// schemes (Table A), 2 for 2nd order (eq. at1) and AT-WENO (eqs. atRecon,
// beta2AT*); AS and SYNC read one level.
int levels_of(int scheme, int mode, int at_levels) {
    if (mode != AT_AT) return 1;
    if (at_levels > 0) return at_levels;
    switch (scheme) {
    case AT_FD2: return 2;
    case AT_FD4: case AT_FD8: return 3;
    case AT_WENO5: case AT_WENO5I: return 2;
    }
    return -1;
}

int kind_of(int pde, int scheme) {
    const bool weno = scheme == AT_WENO5 || scheme == AT_WENO5I;
    switch (pde) {
    case AT_PDE_ADV_DIFF: case AT_PDE_ADR_LOGISTIC: return weno ? K_WSCAL : K_ADR;
    case AT_PDE_BURGERS: return weno ? K_WSCAL : -1;
    case AT_PDE_EULER: return weno ? K_EUL : -1;
    case AT_PDE_REACTIVE_EULER: return weno ? K_REUL : -1;
    case AT_PDE_REACTIVE_NS: return weno ? -1 : K_RNS;
    }
    return -1;
}

static int validate(const at_problem_desc& d, int idx, std::string& err) {
    auto bad = [&](const std::string& m) {
        err = fmt("problem %lld: ", idx) + m;
        return AT_EINVAL;
    };
    if (fields_of(d.pde) < 0) return bad("unknown pde");
    if (halo_of(d.scheme) < 0) return bad("unknown scheme");
    if (d.mode < AT_SYNC || d.mode > AT_AT) return bad("unknown mode");
    if (d.granularity < AT_PER_PE || d.granularity > AT_PER_BOUNDARY) return bad("unknown granularity");
    if (d.precision < AT_FP64 || d.precision > AT_FP32) return bad("unknown precision");
    int S;
    double a[MAXS][MAXS], b[MAXS];
    if (rk_tableau(d.rk, &S, a, b)) return bad("unknown rk");
    if (kind_of(d.pde, d.scheme) < 0) return bad("pde/scheme combination not defined");
    if ((d.pde == AT_PDE_ADV_DIFF || d.pde == AT_PDE_ADR_LOGISTIC) && (d.scheme == AT_WENO5 || d.scheme == AT_WENO5I) &&
        d.alpha != 0.0)
        return bad("WENO5 with diffusion is not defined (alpha must be 0)");
    if (d.n < 1 || d.p < 1 || d.p > d.n) return bad("need 1 <= p <= n");
    if (d.n > (int64_t(1) << 40)) return bad("n too large");
    if (d.kmax < 0 || d.kmax > 15) return bad("kmax must be in 0..15");
    if (d.n_cdf != 0 && d.n_cdf != d.kmax) return bad("n_cdf must be 0 or kmax");
    for (int i = 0; i < d.n_cdf; ++i) {
        if (d.cdf[i] > (uint64_t(1) << 32)) return bad("cdf threshold above 2^32");
        if (i > 0 && d.cdf[i] < d.cdf[i - 1]) return bad("cdf thresholds must not decrease");
    }
    if (d.at_levels < 0 || d.at_levels > 6) return bad("at_levels must be in 0..6");
    if (!(d.dt > 0.0) || !(d.lx > 0.0)) return bad("dt and lx must be positive");
    if (d.bc != 0 && d.bc != 1) return bad("unknown bc");
    if (d.form != 0 && d.form != 1) return bad("unknown form");
    if (d.form == 1 && (d.pde != AT_PDE_REACTIVE_NS || d.bc != 0))
        return bad("the chain-rule form is defined for periodic reactive NS problems");
    return AT_OK;
}

int make_plan(const at_problem_desc* probs, int n_probs, const at_run_opts* opts, Plan& plan,
              std::string& err) {
    if (!probs || n_probs < 1) {
        err = "no problems";
        return AT_EINVAL;
    }
    plan = Plan();
    plan.desc.assign(probs, probs + n_probs);
    std::memset(&plan.opts, 0, sizeof(plan.opts));
    if (opts) plan.opts = *opts;
    if (plan.opts.log_steps < 0 || plan.opts.override_steps < 0 || plan.opts.tile_points < 0 ||
        plan.opts.graph_steps < 0 || plan.opts.grid_per_cu < 0 || plan.opts.lds_budget < 0 ||
        plan.opts.tile_class < 0 || plan.opts.tile_class > 1 || plan.opts.halo_lds < 0 || plan.opts.halo_lds > 1) {
        err = "run option out of range";
        return AT_EINVAL;
    }
    plan.info.resize(n_probs);
    plan.total_points = 0;
    plan.total_pes = 0;
    plan.max_jmax = 1;
    for (int b = 0; b < n_probs; ++b) {
        const at_problem_desc& d = plan.desc[b];
        int rc = validate(d, b, err);
        if (rc) return rc;
        ProbInfo& pi = plan.info[b];
        int S;
        double a[MAXS][MAXS], bw[MAXS];
        rk_tableau(d.rk, &S, a, bw);
        const int kind = kind_of(d.pde, d.scheme);
        const bool f32 = d.precision != AT_FP64;
        // tile class 1: every tile takes the large points-per-thread class
        pi.key = VariantKey{kind, halo_of(d.scheme), S, f32,
                            plan.opts.tile_class == 1 ? ppt_large(kind, f32) : ppt_small(kind, f32)};
        {
            // both tile classes of the combination must be compiled (e.g. the reactive
            // Navier-Stokes kernels exist for the 4th- and 8th-order stencils only)
            VariantKey kl = pi.key;
            kl.ppt = ppt_large(kind, f32);
            int64_t lds, rec;
            if (!variant_sizes(pi.key, 1, 1, 1, &lds, &rec, plan.opts.halo_lds != 0) ||
                !variant_sizes(kl, 1, 1, 1, &lds, &rec, plan.opts.halo_lds != 0)) {
                err = fmt("problem %lld: no compiled kernel for pde %lld with scheme %lld", b, d.pde, d.scheme);
                err += fmt(" and %lld RK stages", S);
                return AT_EUNSUPPORTED;
            }
        }
        pi.F = fields_of(d.pde);
        pi.H = pi.key.H;
        pi.S = S;
        pi.J = levels_of(d.scheme, d.mode, d.at_levels);
        pi.D = d.mode == AT_SYNC ? 1 : d.kmax + pi.J;
        pi.st_elems = (int64_t)pi.F * d.n;
        if (d.n >= ((int64_t)1 << 31)) {
            err = fmt("problem %lld: N = %lld is above the 32-bit point index range", b, (long long)d.n);
            return AT_EUNSUPPORTED;
        }
        // the kernels address each array with 32-bit offsets: every array under 4 GiB
        if (pi.st_elems * (int64_t)MAXS * 8 >= ((int64_t)1 << 32)) {
            err = fmt("problem %lld: F x N = %lld state elements exceed the 32-bit offset range", b,
                      (long long)pi.st_elems);
            return AT_EUNSUPPORTED;
        }
        if (d.bc == 1) {
            // non-periodic ends: the reactive NS kind with central differences; the first
            // and the last PE hold the end closure's four points and the S*H points that
            // keep the boundary windows of the neighbouring PE boundaries off the ends
            if (kind != K_RNS) {
                err = fmt("problem %lld: non-periodic ends need the reactive NS kind", b);
                return AT_EUNSUPPORTED;
            }
            const int64_t need = std::max<int64_t>(4, (int64_t)S * pi.H);
            const int64_t first = d.n / d.p, last = d.n - ((int64_t)(d.p - 1) * d.n) / d.p;
            if (first < need || last < need) {
                err = fmt("problem %lld: non-periodic ends need the first and last PE to hold %lld points", b, need);
                return AT_EUNSUPPORTED;
            }
        }
        pi.pe_base = plan.total_pes;
        plan.total_points += d.n;
        plan.total_pes += d.p;
        plan.max_jmax = std::max(plan.max_jmax, pi.J);
    }

    // ---- tiles: whole PEs packed up to the tile target and the LDS budget; a PE
    //      larger than a small tile gets a tile of the large points-per-thread class ----

    const int64_t lds_hard = 160 * 1024;
    std::vector<std::vector<Tile>> small(n_probs), large(n_probs);
    for (int b = 0; b < n_probs; ++b) {
        const at_problem_desc& d = plan.desc[b];
        ProbInfo& pi = plan.info[b];
        VariantKey ks = pi.key, kl = pi.key;
        // default LDS per tile: 6 workgroups per compute unit for the FP32 scalar FD
        // kernels of halo width up to 2 (whose whole-step kernel is held to 6 waves per
        // SIMD); 40 KiB, 4 workgroups, for the others (two 256-point PEs of the FP32 WENO
        // kinds fit: 38 KB for the reacting Euler kind)
        const int64_t lds_budget = plan.opts.lds_budget > 0 ? plan.opts.lds_budget
                                   : (pi.key.kind == K_ADR && pi.key.f32 && pi.key.H <= 2) ? 26 * 1024
                                                                                           : 40 * 1024;
        kl.ppt = ppt_large(pi.key.kind, pi.key.f32);
        const int tsmall = BLOCK * ks.ppt, tlarge = BLOCK * kl.ppt;
        const int target = plan.opts.tile_points > 0 ? std::min(plan.opts.tile_points, tsmall) : tsmall;
        // PEs are packed up to `pack` points: the target, lowered by default for small
        // workloads so that there are about two tiles per compute unit (256 on MI355X)
        // when the PEs allow it (a tile always takes at least one whole PE)
        const int64_t spread = (plan.total_points + 2 * 256 - 1) / (2 * 256);
        const int pack = plan.opts.tile_points > 0 ? target
                                                   : (int)std::min<int64_t>(target, std::max<int64_t>(1, spread));
        Tile cur{b, 0, 0, 0, 0};
        auto pe_lo = [&](int64_t k) { return (k * d.n) / d.p; };
        for (int64_t k = 0; k < d.p; ++k) {
            const int64_t np = pe_lo(k + 1) - pe_lo(k);
            if (np > tlarge) {
                err = fmt("problem %lld: PE of %lld points exceeds the tile limit %lld", b, np, tlarge);
                return AT_EUNSUPPORTED;
            }
            if (np > target) {
                large[b].push_back(Tile{b, (int32_t)k, 1, (int32_t)np, pe_lo(k)});
                continue;
            }
            bool fits = cur.npe > 0 && cur.npts + np <= pack;
            if (fits) {
                int64_t lds, rec;
                fits = variant_sizes(ks, (int)(cur.npts + np), cur.npe + 1, pi.J, &lds, &rec, plan.opts.halo_lds != 0) &&
                       lds <= lds_budget;
            }
            if (!fits && cur.npe > 0) {
                small[b].push_back(cur);
                cur = Tile{b, 0, 0, 0, 0};
            }
            if (cur.npe == 0) {
                cur.pe0 = (int32_t)k;
                cur.lo = pe_lo(k);
            }
            cur.npe += 1;
            cur.npts += (int32_t)np;
        }
        if (cur.npe > 0) small[b].push_back(cur);
        for (int cls = 0; cls < 2; ++cls)
            for (const Tile& t : (cls ? large[b] : small[b])) {
                int64_t lds, rec;
                if (!variant_sizes(cls ? kl : ks, t.npts, t.npe, pi.J, &lds, &rec, plan.opts.halo_lds != 0)) {
                    err = fmt("problem %lld: kernel variant not compiled", b);
                    return AT_EUNSUPPORTED;
                }
                if (lds > lds_hard) {
                    err = fmt("problem %lld: tile needs %lld bytes of LDS", b, lds);
                    return AT_EUNSUPPORTED;
                }
            }
    }
    for (int b = 0; b < n_probs; ++b) {
        ProbInfo& pi = plan.info[b];
        pi.t0 = (int)plan.tiles_pm.size();
        pi.ntiles_small = (int)small[b].size();
        pi.ntiles = pi.ntiles_small + (int)large[b].size();
        plan.tiles_pm.insert(plan.tiles_pm.end(), small[b].begin(), small[b].end());
        plan.tiles_pm.insert(plan.tiles_pm.end(), large[b].begin(), large[b].end());
    }

    // ---- groups (kernel variants incl. tile class), batched order sorted by cost ----
    auto group_of = [&](const VariantKey& k) {
        for (size_t g = 0; g < plan.groups.size(); ++g)
            if (plan.groups[g].key == k) return (int)g;
        Group g;
        g.key = k;
        g.t0 = g.ntiles = 0;
        g.npts_max = g.npe_max = 0;
        g.jmax = 1;
        g.lds_bytes = 0;
        plan.groups.push_back(g);
        return (int)plan.groups.size() - 1;
    };
    std::vector<std::vector<Tile>> gtiles;
    for (int b = 0; b < n_probs; ++b) {
        ProbInfo& pi = plan.info[b];
        VariantKey kl = pi.key;
        kl.ppt = ppt_large(pi.key.kind, pi.key.f32);
        pi.gid[0] = pi.ntiles_small ? group_of(pi.key) : -1;
        pi.gid[1] = pi.ntiles > pi.ntiles_small ? group_of(kl) : -1;
        gtiles.resize(plan.groups.size());
        for (int i = 0; i < pi.ntiles; ++i) {
            const int cls = i < pi.ntiles_small ? 0 : 1;
            Group& g = plan.groups[pi.gid[cls]];
            g.jmax = std::max(g.jmax, pi.J);
            gtiles[pi.gid[cls]].push_back(plan.tiles_pm[pi.t0 + i]);
        }
    }
    for (size_t gi = 0; gi < plan.groups.size(); ++gi) {
        Group& g = plan.groups[gi];
        std::vector<Tile>& ts = gtiles[gi];
        const int wl = 2 * g.key.S * g.key.H;
        auto cost = [&](const Tile& t) { return (int64_t)t.npts + (int64_t)(t.npe + 1) * wl; };
        std::stable_sort(ts.begin(), ts.end(), [&](const Tile& x, const Tile& y) { return cost(x) > cost(y); });
        g.t0 = (int)plan.tiles_bt.size();
        g.ntiles = (int)ts.size();
        g.lds_bytes = 0;
        for (const Tile& t : ts) {
            g.npts_max = std::max(g.npts_max, t.npts);
            g.npe_max = std::max(g.npe_max, t.npe);
            int64_t lds, rec;
            if (!variant_sizes(g.key, t.npts, t.npe, g.jmax, &lds, &rec, plan.opts.halo_lds != 0)) {   // layouts are per tile
                err = "kernel variant not compiled";
                return AT_EUNSUPPORTED;
            }
            g.lds_bytes = std::max(g.lds_bytes, lds);
        }
        plan.tiles_bt.insert(plan.tiles_bt.end(), ts.begin(), ts.end());
        if (g.lds_bytes > lds_hard) {
            err = fmt("kernel group needs %lld bytes of LDS", g.lds_bytes);
            return AT_EUNSUPPORTED;
        }
    }

    // ---- workspace layout ----
    size_t o = 0;
    plan.off_probs = o; o = align256(o + sizeof(ProbDev) * (size_t)n_probs);
    plan.off_tiles_pm = o; o = align256(o + sizeof(Tile) * plan.tiles_pm.size());
    plan.off_tiles_bt = o; o = align256(o + sizeof(Tile) * plan.tiles_bt.size());
    plan.off_tpd_pm = o; o = align256(o + sizeof(ProbDev) * plan.tiles_pm.size());
    plan.off_tpd_bt = o; o = align256(o + sizeof(ProbDev) * plan.tiles_bt.size());
    plan.off_step = o; o = align256(o + 64);
    plan.peoff.clear();
    plan.peoff.reserve((size_t)(plan.total_pes + n_probs));
    for (int b = 0; b < n_probs; ++b) {
        const at_problem_desc& d = plan.desc[b];
        for (int64_t k = 0; k <= d.p; ++k) plan.peoff.push_back((int32_t)((k * d.n) / d.p));
    }
    plan.off_peoff = o; o = align256(o + sizeof(int32_t) * plan.peoff.size());
    plan.state_bytes_per_step = 0;
    plan.strip_bytes_per_step = 0;
    for (int b = 0; b < n_probs; ++b) {
        const at_problem_desc& d = plan.desc[b];
        ProbInfo& pi = plan.info[b];
        const size_t sl = pi.key.f32 ? 4 : 8;
        const size_t st = sl * (size_t)pi.st_elems;
        for (int w = 0; w < 2; ++w) { pi.off_hi[w] = o; o = align256(o + st); }
        for (int w = 0; w < 2; ++w) {
            pi.off_lo[w] = o;
            if (d.precision == AT_FP32C) o = align256(o + 4 * (size_t)pi.st_elems);
        }
        int64_t lds;
        if (!variant_sizes(pi.key, 1, 1, 1, &lds, &pi.rec_bytes, plan.opts.halo_lds != 0)) {
            err = fmt("problem %lld: kernel variant not compiled", b);
            return AT_EUNSUPPORTED;
        }
        pi.ring_bytes = (int64_t)pi.D * d.p * 2 * pi.rec_bytes;
        if (pi.ring_bytes >= ((int64_t)1 << 32)) {
            err = fmt("problem %lld: strip ring of %lld bytes exceeds the 32-bit offset range", b,
                      (long long)pi.ring_bytes);
            return AT_EUNSUPPORTED;
        }
        pi.off_ring = o; o = align256(o + (size_t)pi.ring_bytes);
        pi.kbuf_len = plan.opts.stage_api ? (int64_t)pi.S * pi.st_elems : 0;
        pi.off_kbuf = o; o = align256(o + sl * (size_t)pi.kbuf_len);
        pi.off_ov = o; o = align256(o + (size_t)plan.opts.override_steps * d.p * 2);
        pi.off_log_d = o; o = align256(o + (size_t)plan.opts.log_steps * d.p * 2);
        pi.off_log_e = o; o = align256(o + (size_t)plan.opts.log_steps * d.p * 2);
        const int64_t per_pt = d.precision == AT_FP64 ? 8 : (d.precision == AT_FP32C ? 8 : 4);
        plan.state_bytes_per_step += 2 * pi.st_elems * per_pt;
        plan.strip_bytes_per_step += (int64_t)d.p * 2 * pi.rec_bytes;
    }
    plan.total = o;
    return AT_OK;
}

void fill_probdev(const Plan& plan, int b, unsigned char* base, ProbDev& P, int64_t ov_step0,
                  int64_t ov_n) {
    const at_problem_desc& d = plan.desc[b];
    const ProbInfo& pi = plan.info[b];
    std::memset(&P, 0, sizeof(P));
    P.n = d.n;
    P.p = d.p;
    P.pde = d.pde;
    P.mode = d.mode;
    P.gran = d.granularity;
    P.kmax = d.kmax;
    P.J = pi.J;
    P.D = pi.D;
    P.n_cdf = d.n_cdf;
    P.keep_lo = d.precision == AT_FP32C;
    P.bc = d.bc;
    P.interp = d.scheme == AT_WENO5I ? 1 : 0;
    P.form = d.form;
    P.S = pi.S;
    P.F = pi.F;
    for (int i = 0; i < 16; ++i) P.cdf[i] = d.cdf[i];
    P.seed = d.seed;
    P.pid = d.problem_id;
    P.dt = d.dt;
    P.inv_dx = (double)d.n / d.lx;
    P.inv_dx2 = P.inv_dx * P.inv_dx;
    P.c = d.c;
    P.alpha = d.alpha;
    P.r = d.r;
    P.gamma = d.gamma;
    P.q = d.q;
    P.ea = d.ea;
    P.b = d.b;
    P.mu = d.mu;
    P.kappa = d.pde == AT_PDE_REACTIVE_NS ? d.mu * d.gamma / ((d.gamma - 1.0) * d.pr) : 0.0;
    P.rhoD = d.pde == AT_PDE_REACTIVE_NS ? d.mu / (d.pr * d.le) : 0.0;
    P.eps = d.weno_eps;
    // scalar FD kind: -c d/dx + alpha d2/dx2 as one stencil on differences u_{i+-o} - u_i
    // (the central weights sum to zero), coefficients of o = 1..H
    for (int o = 0; o < 4; ++o) P.lin_p[o] = P.lin_m[o] = 0.0;
    if (d.scheme != AT_WENO5 && d.scheme != AT_WENO5I) {
        const int H = halo_of(d.scheme);
        for (int o = 1; o <= H; ++o) {
            const double a1 = fd_c1(H, o) * P.inv_dx, a2 = fd_c2(H, o) * P.inv_dx2;
            P.lin_p[o - 1] = -d.c * a1 + d.alpha * a2;
            P.lin_m[o - 1] = d.c * a1 + d.alpha * a2;
        }
    }
    // FP32 copies (round to nearest, as the device's conversions)
    double c0 = 0.0;
    for (int o = 0; o < 4; ++o) {
        P.lpf[o] = (float)P.lin_p[o];
        P.lmf[o] = (float)P.lin_m[o];
        c0 += (double)P.lpf[o] + (double)P.lmf[o];
    }
    P.c0f = (float)c0;
    P.rlf = d.pde == AT_PDE_ADR_LOGISTIC ? (float)d.r : 0.f;
    P.dtf = (float)d.dt;
    P.cf = (float)d.c;
    P.rf = (float)d.r;
    P.alphaf = (float)d.alpha;
    P.inv_dxf = (float)P.inv_dx;
    P.inv_dx2f = (float)P.inv_dx2;
    int S;
    rk_tableau(d.rk, &S, P.a, P.bw);
    for (int w = 0; w < 2; ++w) {
        P.st_hi[w] = base + pi.off_hi[w];
        P.st_lo[w] = d.precision == AT_FP32C ? (void*)(base + pi.off_lo[w]) : nullptr;
    }
    P.ring = base + pi.off_ring;
    P.peoff = (int32_t*)(base + plan.off_peoff) + (pi.pe_base + b);
    P.inv_p = 1.0 / (double)d.p;
    P.rec_bytes = pi.rec_bytes;
    P.kbuf = pi.kbuf_len ? (void*)(base + pi.off_kbuf) : nullptr;
    P.kbuf_len = pi.kbuf_len;
    P.ov = ov_n > 0 ? (uint8_t*)(base + pi.off_ov) : nullptr;
    P.ov_step0 = ov_step0;
    P.ov_n = ov_n;
    P.log_cap = plan.opts.log_steps;
    P.log_drawn = plan.opts.log_steps ? (uint8_t*)(base + pi.off_log_d) : nullptr;
    P.log_eff = plan.opts.log_steps ? (uint8_t*)(base + pi.off_log_e) : nullptr;
}

}  // namespace atk
