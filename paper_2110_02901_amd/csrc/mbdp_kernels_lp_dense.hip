// Dense engine instantiations for BF16 and FP8 E4M3 transition rows (one
// 16-byte load carries 8 or 16 values of a row).

#include "mbdp_engines.h"

namespace mbdp {

template <class T, int EPL>
static SolveFn pick_dense_t(const KParams& p) {
  const int m = p.m;
  // FP8 tiles carry 16 values of V per load: at most 8 rows per pass keep
  // the tile, V and the decode within the registers of 4 waves per SIMD
  if (m >= 16 && T::kType != kFP8) return solve_fn<DenseEngine<16, EPL, T>>(p.task);
  if (m >= 8) return solve_fn<DenseEngine<8, EPL, T>>(p.task);
  if (m >= 4) return solve_fn<DenseEngine<4, EPL, T>>(p.task);
  if (m >= 2) return solve_fn<DenseEngine<2, EPL, T>>(p.task);
  return solve_fn<DenseEngine<1, EPL, T>>(p.task);
}

SolveFn pick_dense_lp(const KParams& p) {
  if (p.vdtype == kBF16) return pick_dense_t<ValBF16, 8>(p);
  if (p.vdtype == kFP8) return pick_dense_t<ValFP8, 16>(p);
  return nullptr;
}

}  // namespace mbdp
