// at_plan.hpp -- host-side planning for libat: validation of the problem
// descriptors, packing of whole PEs into tiles (work items), grouping by kernel
// variant, and the layout of the caller-owned device workspace.  Pure C++ (no
// HIP calls) so that the CPU emulation of the kernels uses the same plan.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/at.h"
#include "at_tile.hpp"

namespace atk {

constexpr int BLOCK = 256;          // threads per workgroup of the tile kernels

struct VariantKey {
    int kind, H, S;
    bool f32;
    int ppt;      // points per thread: tiles of at most BLOCK * ppt points
    bool operator==(const VariantKey& o) const {
        return kind == o.kind && H == o.H && S == o.S && f32 == o.f32 && ppt == o.ppt;
    }
};

// LDS bytes and strip-record bytes of a variant (dispatch over the compiled set).
bool variant_sizes(const VariantKey& v, int npts_max, int npe_max, int jmax, int64_t* lds_bytes,
                   int64_t* rec_bytes, bool halo_lds = false);

struct ProbInfo {
    VariantKey key;           // small-tile variant (ppt_small)
    int F, J, D, S, H;
    int ntiles, t0;            // problem-major tile range [t0, t0 + ntiles)
    int ntiles_small;          // the first ntiles_small tiles are of the small class
    int gid[2];                // group of the small / large tile class (-1: none)
    int64_t st_elems;          // F * N
    size_t off_hi[2], off_lo[2], off_ring, off_kbuf, off_ov, off_log_d, off_log_e;
    int64_t rec_bytes, ring_bytes, kbuf_len;
    int64_t pe_base;           // sum of P over earlier problems
};

struct Group {
    VariantKey key;
    int t0, ntiles;            // range in the batched (group-major) tile array
    int npts_max, npe_max, jmax;
    int64_t lds_bytes;
};

struct Plan {
    std::vector<at_problem_desc> desc;
    at_run_opts opts;
    std::vector<ProbInfo> info;
    std::vector<Tile> tiles_pm;      // problem-major (plain form)
    std::vector<Tile> tiles_bt;      // group-major, cost-sorted (batched form)
    std::vector<Group> groups;
    // workspace
    // off_tpd_*: one copy of its problem's descriptor per tile (same order as the tile
    // lists), so that a workgroup reads its tile and descriptor in one round trip
    size_t off_probs, off_tiles_pm, off_tiles_bt, off_tpd_pm, off_tpd_bt, off_step, total;
    // first point of every PE, floor(p N / P) for p = 0..P, of every problem in turn (problem
    // b's P + 1 entries start at entry pe_base + b); uploaded to off_peoff by the binding
    size_t off_peoff;
    std::vector<int32_t> peoff;
    int64_t total_points, total_pes;
    int64_t state_bytes_per_step, strip_bytes_per_step;
    int max_jmax;
};

// Fills `plan`; returns AT_OK or an error code with a message in `err`.
int make_plan(const at_problem_desc* probs, int n_probs, const at_run_opts* opts, Plan& plan,
              std::string& err);

// Build the device description of problem b for a workspace at `base`.
void fill_probdev(const Plan& plan, int b, unsigned char* base, ProbDev& out, int64_t ov_step0,
                  int64_t ov_n);

// RK tableaus in Butcher form (eq. rk1).
int rk_tableau(int rk, int* S, double a[MAXS][MAXS], double b[MAXS]);

int kind_of(int pde, int scheme);
int halo_of(int scheme);
int levels_of(int scheme, int mode, int at_levels);
int fields_of(int pde);

}  // namespace atk
