// at_variants.hpp -- the compiled set of tile-kernel variants: kind, halo width
// H, RK stages S, FP32 form, and points per thread (PPT; a tile holds at most
// 256 * PPT points, so each variant comes in a small and a large tile class).
// One X-macro list shared by the kernels, the planner and the CPU emulation.
#pragma once
#include "at_tile.hpp"

namespace atk {
// points-per-thread classes of each kind and precision: small (default tiles) and
// large (big PEs).  The scalar FD kind takes 8 points per thread in the FP32 forms and
// 6 in FP64 (its state is twice the registers); its large class holds PEs of up to
// 4096 points.
constexpr int ppt_small(int kind, bool f32) {
    return kind == K_ADR ? (f32 ? 8 : 6) : kind == K_WSCAL ? 4 : 2;
}
constexpr int ppt_large(int kind, bool f32) { return kind == K_ADR ? 16 : 2 * ppt_small(kind, f32); }
}  // namespace atk

#define AT_VARIANTS_P(X, K, H, S, F32) \
    X(K, H, S, F32, atk::ppt_small(K, F32)) X(K, H, S, F32, atk::ppt_large(K, F32))
#define AT_VARIANTS_S(X, K, H, F32) \
    AT_VARIANTS_P(X, K, H, 1, F32) AT_VARIANTS_P(X, K, H, 2, F32) AT_VARIANTS_P(X, K, H, 3, F32) \
    AT_VARIANTS_P(X, K, H, 4, F32)
#define AT_VARIANTS_SF(X, K, H) AT_VARIANTS_S(X, K, H, 0) AT_VARIANTS_S(X, K, H, 1)

// the FD kinds in two units each (FP64 / FP32 forms) to halve their compile time
#define AT_VARIANTS_ADR64(X) AT_VARIANTS_S(X, atk::K_ADR, 1, 0) AT_VARIANTS_S(X, atk::K_ADR, 2, 0) \
    AT_VARIANTS_S(X, atk::K_ADR, 4, 0)
#define AT_VARIANTS_ADR32(X) AT_VARIANTS_S(X, atk::K_ADR, 1, 1) AT_VARIANTS_S(X, atk::K_ADR, 2, 1) \
    AT_VARIANTS_S(X, atk::K_ADR, 4, 1)
#define AT_VARIANTS_ADR(X) AT_VARIANTS_ADR64(X) AT_VARIANTS_ADR32(X)
#define AT_VARIANTS_RNS64(X) AT_VARIANTS_S(X, atk::K_RNS, 2, 0) AT_VARIANTS_S(X, atk::K_RNS, 4, 0)
#define AT_VARIANTS_RNS32(X) AT_VARIANTS_S(X, atk::K_RNS, 2, 1) AT_VARIANTS_S(X, atk::K_RNS, 4, 1)
#define AT_VARIANTS_RNS(X) AT_VARIANTS_RNS64(X) AT_VARIANTS_RNS32(X)
#define AT_VARIANTS_WSCAL(X) AT_VARIANTS_SF(X, atk::K_WSCAL, 3)
#define AT_VARIANTS_EUL(X) AT_VARIANTS_SF(X, atk::K_EUL, 3)
#define AT_VARIANTS_REUL(X) AT_VARIANTS_SF(X, atk::K_REUL, 3)

#define AT_VARIANTS(X) AT_VARIANTS_ADR(X) AT_VARIANTS_RNS(X) AT_VARIANTS_WSCAL(X) \
    AT_VARIANTS_EUL(X) AT_VARIANTS_REUL(X)

#define AT_CFG(K, H, S, F32, PPT) atk::Cfg<K, H, S, (F32) != 0, PPT>
