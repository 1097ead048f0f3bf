// ELL engine instantiations for BF16 and FP8 E4M3 values (rows of at most
// 64 entries; each lane holds 4 columns and their 4 values).

#include "mbdp_engines.h"

namespace mbdp {

template <class T>
static SolveFn pick_ell_t(int lpr, bool two, int task) {
  switch (lpr) {
    case 1: return two ? solve_fn<EllEngine<2, 1, T>>(task) : solve_fn<EllEngine<1, 1, T>>(task);
    case 2: return two ? solve_fn<EllEngine<2, 2, T>>(task) : solve_fn<EllEngine<1, 2, T>>(task);
    case 4: return two ? solve_fn<EllEngine<2, 4, T>>(task) : solve_fn<EllEngine<1, 4, T>>(task);
    case 8: return two ? solve_fn<EllEngine<2, 8, T>>(task) : solve_fn<EllEngine<1, 8, T>>(task);
    case 16:
      return two ? solve_fn<EllEngine<2, 16, T>>(task) : solve_fn<EllEngine<1, 16, T>>(task);
    default: return nullptr;
  }
}

SolveFn pick_ell_lp(const KParams& p, int units_per_wave_hint) {
  int lpr = 1;
  while (lpr * 4 < p.ell_k) lpr <<= 1;
  const bool two = units_per_wave_hint >= 2;
  if (p.vdtype == kBF16) return pick_ell_t<ValBF16>(lpr, two, p.task);
  if (p.vdtype == kFP8) return pick_ell_t<ValFP8>(lpr, two, p.task);
  return nullptr;
}

}  // namespace mbdp
