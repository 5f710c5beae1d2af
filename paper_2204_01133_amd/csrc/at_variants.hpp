// at_variants.hpp -- the compiled set of tile-kernel variants (kind, halo width
// H, RK stages S, FP32 form).  One X-macro list shared by the kernels, the
// planner's size queries and the CPU emulation.
#pragma once
#include "at_tile.hpp"

namespace atk {
constexpr int ppt_c(int kind) { return (kind == K_ADR || kind == K_WSCAL) ? 8 : 4; }
}  // namespace atk

#define AT_VARIANTS_SF(X, K, H) \
    X(K, H, 1, 0) X(K, H, 2, 0) X(K, H, 3, 0) X(K, H, 4, 0) \
    X(K, H, 1, 1) X(K, H, 2, 1) X(K, H, 3, 1) X(K, H, 4, 1)

#define AT_VARIANTS_ADR(X) AT_VARIANTS_SF(X, atk::K_ADR, 1) AT_VARIANTS_SF(X, atk::K_ADR, 2) \
    AT_VARIANTS_SF(X, atk::K_ADR, 4)
#define AT_VARIANTS_RNS(X) AT_VARIANTS_SF(X, atk::K_RNS, 2) AT_VARIANTS_SF(X, atk::K_RNS, 4)
#define AT_VARIANTS_WSCAL(X) AT_VARIANTS_SF(X, atk::K_WSCAL, 3)
#define AT_VARIANTS_EUL(X) AT_VARIANTS_SF(X, atk::K_EUL, 3)
#define AT_VARIANTS_REUL(X) AT_VARIANTS_SF(X, atk::K_REUL, 3)

#define AT_VARIANTS(X) AT_VARIANTS_ADR(X) AT_VARIANTS_RNS(X) AT_VARIANTS_WSCAL(X) \
    AT_VARIANTS_EUL(X) AT_VARIANTS_REUL(X)

#define AT_CFG(K, H, S, F32) atk::Cfg<K, H, S, (F32) != 0, atk::ppt_c(K)>
