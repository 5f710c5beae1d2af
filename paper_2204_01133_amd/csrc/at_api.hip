// at_api.hip -- libat's C ABI (include/at.h) on HIP: planning, the caller-owned
// workspace, state conversion kernels, the plain / batched / per-stage step
// launches and HIP-graph replay of batched steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/at.h"
#include "at_kernels.hpp"
#include "at_plan.hpp"

using namespace atk;

struct at_ctx {
    Plan plan;
    std::string err;
    unsigned char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    bool bound = false;
    int64_t step = 0;
    int stage = 0;
    std::vector<uint8_t> state_set;
    std::vector<int64_t> ov_step0, ov_n;
    std::vector<ProbDev> pd;
    std::vector<ProbDev> tpd_pm, tpd_bt;   // per-tile descriptor copies (host staging)
    int num_cus = 256;
    // the groups of a batched step run concurrently: group 0 on the caller's stream, every
    // other group on a stream of its own, forked from and joined back into the caller's
    // stream with events (fork event first, then one join event per side stream)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;
    // graph of graph_steps batched steps
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int graph_len = 0;
    // bound to the library's device scratch (at_bind_scratch) on this device, else -1
    int scratch_dev = -1;
};

// Device scratch for callers that cannot allocate device memory (at_bind_scratch): a
// file-scope device array, one copy per device, held until the process ends.  Host code
// never uses its name as an address: the device address of each device's copy is looked
// up once per device (hipGetSymbolAddress, with that device current) and kept here.
// (AT_SCRATCH_BYTES, the array's size, is part of the C ABI: include/at.h)
static __device__ __align__(256) unsigned char scratch[AT_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEV = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEV] = {};
const at_ctx* g_scratch_owner[SCRATCH_MAX_DEV] = {};

int fail(at_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(at_ctx* c, hipError_t e, const char* where) {
    return fail(c, AT_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, expr)                                          \
    do {                                                         \
        hipError_t _e = (expr);                                  \
        if (_e != hipSuccess) return hip_fail((c), _e, #expr);   \
    } while (0)

__global__ void k_split(const double* __restrict__ q, float* __restrict__ hi, float* __restrict__ lo,
                        int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = q[i];
    const float h = (float)v;
    hi[i] = h;
    if (lo) lo[i] = (float)(v - (double)h);
}

__global__ void k_join(const float* __restrict__ hi, const float* __restrict__ lo, double* __restrict__ out,
                       int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = (double)hi[i] + (lo ? (double)lo[i] : 0.0);
}

__global__ void k_set_step(int64_t* d, int64_t v) { *d = v; }
__global__ void k_add_step(int64_t* d, int64_t v) { *d += v; }

int launch_key(at_ctx* c, const VariantKey& k, const KArgs& a, int grid, hipStream_t s) {
    if (grid <= 0 || a.ntiles <= 0) return AT_OK;
    hipError_t e = hipSuccess;
    bool ok = launch_adr(k, a, grid, s, &e) || launch_adr32(k, a, grid, s, &e) ||
              launch_rns(k, a, grid, s, &e) || launch_rns32(k, a, grid, s, &e) ||
              launch_wscal(k, a, grid, s, &e) || launch_eul(k, a, grid, s, &e) ||
              launch_reul(k, a, grid, s, &e);
    if (!ok) return fail(c, AT_EUNSUPPORTED, "kernel variant not compiled");
    if (e != hipSuccess) return hip_fail(c, e, "tile kernel launch");
    return AT_OK;
}

KArgs base_args(at_ctx* c, const Group& g) {
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.probs = (const ProbDev*)(c->ws + c->plan.off_probs);
    a.npts_max = g.npts_max;
    a.npe_max = g.npe_max;
    a.jmax = g.jmax;
    a.lds_bytes = (int32_t)g.lds_bytes;
    a.flags = (c->plan.opts.log_steps ? KF_LOG : 0) | (c->plan.opts.xcd_remap ? KF_XCD : 0) |
              (c->plan.opts.halo_lds ? KF_HALO_LDS : 0);
    return a;
}

int upload_probs(at_ctx* c) {
    for (size_t b = 0; b < c->plan.desc.size(); ++b)
        fill_probdev(c->plan, (int)b, c->ws, c->pd[b], c->ov_step0[b], c->ov_n[b]);
    HIPCHK(c, hipMemcpyAsync(c->ws + c->plan.off_probs, c->pd.data(), sizeof(ProbDev) * c->pd.size(),
                             hipMemcpyHostToDevice, c->stream));
    for (int w = 0; w < 2; ++w) {
        const std::vector<Tile>& tl = w ? c->plan.tiles_bt : c->plan.tiles_pm;
        std::vector<ProbDev>& tp = w ? c->tpd_bt : c->tpd_pm;
        tp.resize(tl.size());
        for (size_t i = 0; i < tl.size(); ++i) tp[i] = c->pd[tl[i].prob];
        HIPCHK(c, hipMemcpyAsync(c->ws + (w ? c->plan.off_tpd_bt : c->plan.off_tpd_pm), tp.data(),
                                 sizeof(ProbDev) * tp.size(), hipMemcpyHostToDevice, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return AT_OK;
}

// bound, and (for the device scratch) still the context that holds it
int check_bound(at_ctx* c) {
    if (!c->bound) return fail(c, AT_ESTATE, "workspace not bound");
    if (c->scratch_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (g_scratch_owner[c->scratch_dev] != c)
            return fail(c, AT_ESTATE, "the device scratch was bound to another context since");
    }
    return AT_OK;
}

int check_ready(at_ctx* c) {
    if (!c) return AT_EINVAL;
    if (int rb = check_bound(c)) return rb;
    for (size_t b = 0; b < c->state_set.size(); ++b)
        if (!c->state_set[b]) return fail(c, AT_ESTATE, "state of a problem not set");
    return AT_OK;
}

// side streams and events for concurrent groups (created once per context)
int make_side_streams(at_ctx* c) {
    const size_t ng = c->plan.groups.size();
    while (c->side.size() + 1 < ng) {
        hipStream_t st = nullptr;
        HIPCHK(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        c->side.push_back(st);
    }
    while (ng > 1 && c->ev.size() < ng) {
        hipEvent_t e = nullptr;
        HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->ev.push_back(e);
    }
    return AT_OK;
}

void free_side_streams(at_ctx* c) {
    for (hipStream_t st : c->side) (void)hipStreamDestroy(st);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->side.clear();
    c->ev.clear();
}

// one batched step (all groups, all stages) with step counter n or from the device counter.
// The tiles of a step are independent (they read level n and older, and write level n+1
// and their own ring records of level n), so the groups run concurrently.
int batched_step_launches(at_ctx* c, const int64_t* step_ptr, int64_t step_off) {
    const size_t ng = c->plan.groups.size();
    // bound to the device scratch: no side streams or events, the groups run one after
    // another on the context's stream
    const bool concurrent = ng > 1 && c->scratch_dev < 0;
    if (concurrent) {
        if (c->side.size() + 1 < ng || c->ev.size() < ng) return fail(c, AT_ESTATE, "side streams missing");
        HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
        for (size_t i = 1; i < ng; ++i) HIPCHK(c, hipStreamWaitEvent(c->side[i - 1], c->ev[0], 0));
    }
    for (size_t gi = 0; gi < ng; ++gi) {
        const Group& g = c->plan.groups[gi];
        KArgs a = base_args(c, g);
        a.tiles = (const Tile*)(c->ws + c->plan.off_tiles_bt) + g.t0;
        a.tprobs = (const ProbDev*)(c->ws + c->plan.off_tpd_bt) + g.t0;
        a.ntiles = g.ntiles;
        a.step_ptr = step_ptr;
        a.step_off = step_off;
        a.s_begin = 0;
        a.s_end = g.key.S - 1;
        // the planner's choice is one workgroup per tile: with whole tiles per workgroup
        // and several workgroups per CU it measured faster than a persistent grid on
        // every configuration (C3: 0.075 against 0.078-0.081 ms per step)
        const int persistent = c->plan.opts.persistent == 1 ? 1 : 0;
        const int per_cu = c->plan.opts.grid_per_cu > 0 ? c->plan.opts.grid_per_cu : 6;
        const int grid = persistent ? std::min(g.ntiles, per_cu * c->num_cus) : g.ntiles;
        int rc = launch_key(c, g.key, a, grid, (gi == 0 || !concurrent) ? c->stream : c->side[gi - 1]);
        if (rc) return rc;
    }
    for (size_t i = 1; concurrent && i < ng; ++i) {
        HIPCHK(c, hipEventRecord(c->ev[i], c->side[i - 1]));
        HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev[i], 0));
    }
    return AT_OK;
}

void drop_graph(at_ctx* c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->graph_len = 0;
}

int build_graph(at_ctx* c, int len) {
    drop_graph(c);
    int64_t* d_step = (int64_t*)(c->ws + c->plan.off_step);
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = AT_OK;
    for (int k = 0; k < len && rc == AT_OK; ++k) rc = batched_step_launches(c, d_step, k);
    if (rc == AT_OK) hipLaunchKernelGGL(k_add_step, dim3(1), dim3(1), 0, c->stream, d_step, (int64_t)len);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    c->graph = g;
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(c);
        return hip_fail(c, e, "hipGraphInstantiate");
    }
    c->graph_len = len;
    return AT_OK;
}

}  // namespace

extern "C" {

// the planner's message of the calling thread's last failed at_init
thread_local std::string g_init_err;

int at_init(const at_problem_desc* probs, int n_probs, const at_run_opts* opts, at_ctx** out,
            size_t* workspace_bytes) {
    g_init_err.clear();
    if (!out || !workspace_bytes) {
        g_init_err = "null output argument";
        return AT_EINVAL;
    }
    *out = nullptr;
    at_ctx* c = new at_ctx();
    int rc = make_plan(probs, n_probs, opts, c->plan, c->err);
    if (rc) {
        g_init_err = c->err;                 // for at_last_error(NULL) on this thread
        delete c;
        return rc;
    }
    c->state_set.assign(n_probs, 0);
    c->ov_step0.assign(n_probs, 0);
    c->ov_n.assign(n_probs, 0);
    c->pd.resize(n_probs);
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            c->num_cus = cus;
    }
    *workspace_bytes = c->plan.total;
    *out = c;
    return AT_OK;
}

namespace {
void release_scratch(at_ctx* c) {
    if (c->scratch_dev < 0) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_owner[c->scratch_dev] == c) g_scratch_owner[c->scratch_dev] = nullptr;
    c->scratch_dev = -1;
}
}  // namespace

int at_bind(at_ctx* c, void* d_workspace, size_t bytes, void* hip_stream) {
    if (!c || !d_workspace) return AT_EINVAL;
    if (bytes < c->plan.total) return fail(c, AT_EINVAL, "workspace too small");
    if (((uintptr_t)d_workspace & 255) != 0) return fail(c, AT_EINVAL, "workspace not 256-byte aligned");
    release_scratch(c);
    drop_graph(c);
    c->step = 0;
    c->stage = 0;
    std::fill(c->state_set.begin(), c->state_set.end(), 0);
    c->ws = (unsigned char*)d_workspace;
    c->ws_bytes = bytes;
    c->stream = (hipStream_t)hip_stream;
    HIPCHK(c, hipMemcpyAsync(c->ws + c->plan.off_tiles_pm, c->plan.tiles_pm.data(),
                             sizeof(Tile) * c->plan.tiles_pm.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ws + c->plan.off_tiles_bt, c->plan.tiles_bt.data(),
                             sizeof(Tile) * c->plan.tiles_bt.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ws + c->plan.off_peoff, c->plan.peoff.data(),
                             sizeof(int32_t) * c->plan.peoff.size(), hipMemcpyHostToDevice, c->stream));
    int rc = make_side_streams(c);
    if (rc) return rc;
    c->bound = true;
    return upload_probs(c);
}

int at_bind_scratch(at_ctx* c, void* hip_stream) {
    if (!c) return AT_EINVAL;
    if (c->plan.total > AT_SCRATCH_BYTES)
        return fail(c, AT_EUNSUPPORTED,
                    "workspace of " + std::to_string(c->plan.total) + " bytes exceeds the device scratch of " +
                        std::to_string(AT_SCRATCH_BYTES) + " bytes (use at_bind with a caller-owned workspace)");
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEV) return fail(c, AT_EUNSUPPORTED, "device index beyond the scratch table");
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            // the device address of this device's copy of the array (the current device)
            hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
            if (!ptr || ((uintptr_t)ptr & 255) != 0) return fail(c, AT_EHIP, "device scratch not 256-byte aligned");
            g_scratch_ptr[dev] = ptr;
        }
        ptr = g_scratch_ptr[dev];
    }
    release_scratch(c);
    drop_graph(c);
    c->step = 0;
    c->stage = 0;
    std::fill(c->state_set.begin(), c->state_set.end(), 0);
    c->ws = (unsigned char*)ptr;
    c->ws_bytes = AT_SCRATCH_BYTES;
    c->stream = (hipStream_t)hip_stream;
    c->bound = false;
    HIPCHK(c, hipMemcpyAsync(c->ws + c->plan.off_tiles_pm, c->plan.tiles_pm.data(),
                             sizeof(Tile) * c->plan.tiles_pm.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ws + c->plan.off_tiles_bt, c->plan.tiles_bt.data(),
                             sizeof(Tile) * c->plan.tiles_bt.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->ws + c->plan.off_peoff, c->plan.peoff.data(),
                             sizeof(int32_t) * c->plan.peoff.size(), hipMemcpyHostToDevice, c->stream));
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        g_scratch_owner[dev] = c;
    }
    c->scratch_dev = dev;
    c->bound = true;
    return upload_probs(c);
}

int at_reset(at_ctx* c) {
    if (!c) return AT_EINVAL;
    c->step = 0;
    c->stage = 0;
    std::fill(c->state_set.begin(), c->state_set.end(), 0);
    return AT_OK;
}

int at_set_state(at_ctx* c, int prob, const double* q, int q_on_device) {
    if (!c || !q) return AT_EINVAL;
    if (int rb = check_bound(c)) return rb;
    if (prob < 0 || prob >= (int)c->plan.desc.size()) return fail(c, AT_EINVAL, "problem index");
    if (c->step != 0 || c->stage != 0) return fail(c, AT_ESTATE, "state set after stepping (at_reset first)");
    const ProbInfo& pi = c->plan.info[prob];
    const int prec = c->plan.desc[prob].precision;
    const int64_t n = pi.st_elems;
    if (prec == AT_FP64) {
        HIPCHK(c, hipMemcpyAsync(c->ws + pi.off_hi[0], q, 8 * (size_t)n,
                                 q_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
        if (!q_on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
    } else if (q_on_device) {
        float* lo = prec == AT_FP32C ? (float*)(c->ws + pi.off_lo[0]) : nullptr;
        hipLaunchKernelGGL(k_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, q,
                           (float*)(c->ws + pi.off_hi[0]), lo, n);
        HIPCHK(c, hipGetLastError());
    } else {
        std::vector<float> hi(n), lo(n);
        for (int64_t i = 0; i < n; ++i) {
            hi[i] = (float)q[i];
            lo[i] = (float)(q[i] - (double)hi[i]);
        }
        HIPCHK(c, hipMemcpyAsync(c->ws + pi.off_hi[0], hi.data(), 4 * (size_t)n, hipMemcpyHostToDevice, c->stream));
        if (prec == AT_FP32C)
            HIPCHK(c, hipMemcpyAsync(c->ws + pi.off_lo[0], lo.data(), 4 * (size_t)n, hipMemcpyHostToDevice,
                                     c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->state_set[prob] = 1;
    return AT_OK;
}

int at_step(at_ctx* c, int n_steps) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (c->stage != 0) return fail(c, AT_ESTATE, "at_step inside a per-stage step");
    if (n_steps < 0) return fail(c, AT_EINVAL, "negative step count");
    for (int i = 0; i < n_steps; ++i) {
        for (size_t b = 0; b < c->plan.desc.size(); ++b) {
            const ProbInfo& pi = c->plan.info[b];
            for (int cls = 0; cls < 2; ++cls) {
                if (pi.gid[cls] < 0) continue;
                const Group& g = c->plan.groups[pi.gid[cls]];
                KArgs a = base_args(c, g);
                const int off = cls ? pi.ntiles_small : 0;
                const int cnt = cls ? pi.ntiles - pi.ntiles_small : pi.ntiles_small;
                a.tiles = (const Tile*)(c->ws + c->plan.off_tiles_pm) + pi.t0 + off;
                a.tprobs = (const ProbDev*)(c->ws + c->plan.off_tpd_pm) + pi.t0 + off;
                a.ntiles = cnt;
                a.step_off = c->step;
                a.s_begin = 0;
                a.s_end = pi.S - 1;
                rc = launch_key(c, g.key, a, cnt, c->stream);
                if (rc) return rc;
            }
        }
        c->step += 1;
    }
    return AT_OK;
}

int at_batch_step(at_ctx* c, int n_steps) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (c->stage != 0) return fail(c, AT_ESTATE, "at_batch_step inside a per-stage step");
    if (n_steps < 0) return fail(c, AT_EINVAL, "negative step count");
    // bound to the device scratch: plain launches only (instantiating a graph may allocate)
    const int gl = c->scratch_dev >= 0 ? 0 : c->plan.opts.graph_steps;
    int done = 0;
    if (gl > 0 && c->stream != nullptr && n_steps >= gl) {
        if (!c->gexec || c->graph_len != gl) {
            rc = build_graph(c, gl);
            if (rc) return rc;
        }
        int64_t* d_step = (int64_t*)(c->ws + c->plan.off_step);
        hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, c->stream, d_step, c->step);
        HIPCHK(c, hipGetLastError());
        while (n_steps - done >= gl) {
            HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
            done += gl;
            c->step += gl;
        }
    }
    for (; done < n_steps; ++done) {
        rc = batched_step_launches(c, nullptr, c->step);
        if (rc) return rc;
        c->step += 1;
    }
    return AT_OK;
}

int at_rk_stage(at_ctx* c, int stage) {
    int rc = check_ready(c);
    if (rc) return rc;
    if (!c->plan.opts.stage_api) return fail(c, AT_ESTATE, "stage buffers not reserved (stage_api)");
    const int S = c->plan.info[0].S;
    for (const ProbInfo& pi : c->plan.info)
        if (pi.S != S) return fail(c, AT_EUNSUPPORTED, "per-stage stepping needs one RK scheme");
    if (stage != c->stage + 1 || stage < 1 || stage > S)
        return fail(c, AT_ESTATE, "stages must be called in order 1..S");
    for (const Group& g : c->plan.groups) {
        KArgs a = base_args(c, g);
        a.tiles = (const Tile*)(c->ws + c->plan.off_tiles_bt) + g.t0;
        a.tprobs = (const ProbDev*)(c->ws + c->plan.off_tpd_bt) + g.t0;
        a.ntiles = g.ntiles;
        a.step_off = c->step;
        a.s_begin = stage - 1;
        a.s_end = stage - 1;
        a.flags |= KF_STAGE_IO;
        rc = launch_key(c, g.key, a, g.ntiles, c->stream);
        if (rc) return rc;
    }
    c->stage = stage;
    if (stage == S) {
        c->stage = 0;
        c->step += 1;
    }
    return AT_OK;
}

int at_get_state(at_ctx* c, int prob, double* out, int out_on_device) {
    if (!c || !out) return AT_EINVAL;
    if (int rb = check_bound(c)) return rb;
    if (prob < 0 || prob >= (int)c->plan.desc.size()) return fail(c, AT_EINVAL, "problem index");
    const ProbInfo& pi = c->plan.info[prob];
    const int prec = c->plan.desc[prob].precision;
    const int w = (int)(c->step & 1);
    const int64_t n = pi.st_elems;
    if (prec == AT_FP64) {
        HIPCHK(c, hipMemcpyAsync(out, c->ws + pi.off_hi[w], 8 * (size_t)n,
                                 out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    } else if (out_on_device) {
        const float* lo = prec == AT_FP32C ? (const float*)(c->ws + pi.off_lo[w]) : nullptr;
        hipLaunchKernelGGL(k_join, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                           (const float*)(c->ws + pi.off_hi[w]), lo, out, n);
        HIPCHK(c, hipGetLastError());
    } else {
        std::vector<float> hi(n), lo(n, 0.f);
        HIPCHK(c, hipMemcpyAsync(hi.data(), c->ws + pi.off_hi[w], 4 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
        if (prec == AT_FP32C)
            HIPCHK(c, hipMemcpyAsync(lo.data(), c->ws + pi.off_lo[w], 4 * (size_t)n, hipMemcpyDeviceToHost,
                                     c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int64_t i = 0; i < n; ++i) out[i] = (double)hi[i] + (double)lo[i];
        return AT_OK;
    }
    if (!out_on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
    return AT_OK;
}

int at_get_delays(at_ctx* c, int prob, int64_t step0, int n_steps, uint8_t* drawn, uint8_t* eff) {
    if (!c || !drawn || !eff) return AT_EINVAL;
    if (int rb = check_bound(c)) return rb;
    if (prob < 0 || prob >= (int)c->plan.desc.size()) return fail(c, AT_EINVAL, "problem index");
    const int64_t cap = c->plan.opts.log_steps;
    if (cap == 0) return fail(c, AT_EINVAL, "delay log disabled (log_steps = 0)");
    if (n_steps < 0 || step0 < 0 || step0 + n_steps > c->step || step0 < c->step - cap)
        return fail(c, AT_ERANGE, "steps outside the logged window");
    const ProbInfo& pi = c->plan.info[prob];
    const int64_t P = c->plan.desc[prob].p;
    for (int i = 0; i < n_steps; ++i) {
        const int64_t slot = (step0 + i) % cap;
        HIPCHK(c, hipMemcpyAsync(drawn + (int64_t)i * P * 2, c->ws + pi.off_log_d + slot * P * 2, (size_t)P * 2,
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(eff + (int64_t)i * P * 2, c->ws + pi.off_log_e + slot * P * 2, (size_t)P * 2,
                                 hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return AT_OK;
}

int at_set_delay_override(at_ctx* c, int prob, const uint8_t* sched, int64_t step0, int n_steps) {
    if (!c) return AT_EINVAL;
    if (int rb = check_bound(c)) return rb;
    if (prob < 0 || prob >= (int)c->plan.desc.size()) return fail(c, AT_EINVAL, "problem index");
    if (n_steps < 0 || step0 < 0) return fail(c, AT_EINVAL, "negative step");
    if (n_steps > c->plan.opts.override_steps) return fail(c, AT_EINVAL, "schedule longer than override_steps");
    if (n_steps > 0 && !sched) return AT_EINVAL;
    const int64_t P = c->plan.desc[prob].p;
    for (int64_t i = 0; i < (int64_t)n_steps * P * 2; ++i)
        if (sched[i] > c->plan.desc[prob].kmax)
            return fail(c, AT_ESTALE, "override delay above kmax: the ring holds kmax + J levels");
    if (n_steps > 0) {
        HIPCHK(c, hipMemcpyAsync(c->ws + c->plan.info[prob].off_ov, sched, (size_t)n_steps * P * 2,
                                 hipMemcpyHostToDevice, c->stream));
    }
    c->ov_step0[prob] = step0;
    c->ov_n[prob] = n_steps;
    return upload_probs(c);
}

int at_sync(at_ctx* c) {
    if (!c) return AT_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return AT_OK;
}

int at_query(const at_ctx* c, int key, int64_t* v) {
    if (!c || !v) return AT_EINVAL;
    switch (key) {
    case AT_Q_STEP: *v = c->step; return AT_OK;
    case AT_Q_NUM_TILES: *v = (int64_t)c->plan.tiles_bt.size(); return AT_OK;
    case AT_Q_NUM_GROUPS: *v = (int64_t)c->plan.groups.size(); return AT_OK;
    case AT_Q_TOTAL_POINTS: *v = c->plan.total_points; return AT_OK;
    case AT_Q_STATE_BYTES: *v = c->plan.state_bytes_per_step; return AT_OK;
    case AT_Q_STAGES: *v = c->plan.info[0].S; return AT_OK;
    case AT_Q_LDS_BYTES: {
        int64_t m = 0;
        for (const Group& g : c->plan.groups) m = std::max(m, g.lds_bytes);
        *v = m;
        return AT_OK;
    }
    case AT_Q_STRIP_BYTES: *v = c->plan.strip_bytes_per_step; return AT_OK;
    case AT_Q_NUM_PES: *v = c->plan.total_pes; return AT_OK;
    }
    return AT_EINVAL;
}

void* at_stream(const at_ctx* c) { return c ? (void*)c->stream : nullptr; }

const char* at_strerror(int code) {
    switch (code) {
    case AT_OK: return "ok";
    case AT_EINVAL: return "invalid argument";
    case AT_EUNSUPPORTED: return "unsupported";
    case AT_ESTATE: return "wrong call order";
    case AT_EHIP: return "HIP error";
    case AT_ESTALE: return "delay older than the ring holds";
    case AT_ERANGE: return "out of range";
    }
    return "unknown error";
}

const char* at_last_error(const at_ctx* c) { return c ? c->err.c_str() : g_init_err.c_str(); }

void at_free(at_ctx* c) {
    if (!c) return;
    release_scratch(c);
    drop_graph(c);
    free_side_streams(c);
    delete c;
}

}  // extern "C"
