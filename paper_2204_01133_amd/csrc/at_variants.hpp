// at_variants.hpp -- the compiled set of tile-kernel variants: kind, halo width
// H, RK stages S, FP32 form, and points per thread (PPT; a tile holds at most
// 256 * PPT points, so each variant comes in a small and a large tile class).
// One X-macro list shared by the kernels, the planner and the CPU emulation.
#pragma once
#include "at_tile.hpp"

namespace atk {
// points-per-thread classes of each kind: small (default tiles) and large (big PEs)
constexpr int ppt_small(int kind) { return kind == K_ADR ? 8 : kind == K_WSCAL ? 4 : 2; }
constexpr int ppt_large(int kind) { return kind == K_ADR ? 16 : kind == K_WSCAL ? 8 : 4; }
}  // namespace atk

#define AT_VARIANTS_P(X, K, H, S, F32) X(K, H, S, F32, atk::ppt_small(K)) X(K, H, S, F32, atk::ppt_large(K))
#define AT_VARIANTS_SF(X, K, H) \
    AT_VARIANTS_P(X, K, H, 1, 0) AT_VARIANTS_P(X, K, H, 2, 0) AT_VARIANTS_P(X, K, H, 3, 0) \
    AT_VARIANTS_P(X, K, H, 4, 0) AT_VARIANTS_P(X, K, H, 1, 1) AT_VARIANTS_P(X, K, H, 2, 1) \
    AT_VARIANTS_P(X, K, H, 3, 1) AT_VARIANTS_P(X, K, H, 4, 1)

#define AT_VARIANTS_ADR(X) AT_VARIANTS_SF(X, atk::K_ADR, 1) AT_VARIANTS_SF(X, atk::K_ADR, 2) \
    AT_VARIANTS_SF(X, atk::K_ADR, 4)
#define AT_VARIANTS_RNS(X) AT_VARIANTS_SF(X, atk::K_RNS, 2) AT_VARIANTS_SF(X, atk::K_RNS, 4)
#define AT_VARIANTS_WSCAL(X) AT_VARIANTS_SF(X, atk::K_WSCAL, 3)
#define AT_VARIANTS_EUL(X) AT_VARIANTS_SF(X, atk::K_EUL, 3)
#define AT_VARIANTS_REUL(X) AT_VARIANTS_SF(X, atk::K_REUL, 3)

#define AT_VARIANTS(X) AT_VARIANTS_ADR(X) AT_VARIANTS_RNS(X) AT_VARIANTS_WSCAL(X) \
    AT_VARIANTS_EUL(X) AT_VARIANTS_REUL(X)

#define AT_CFG(K, H, S, F32, PPT) atk::Cfg<K, H, S, (F32) != 0, PPT>
