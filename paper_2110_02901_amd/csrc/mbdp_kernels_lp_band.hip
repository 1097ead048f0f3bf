// Band-local ELL engine instantiations for BF16 and FP8 E4M3 values (rows of
// at most 64 entries).

#include "mbdp_engines.h"

namespace mbdp {

template <class T>
static SolveFn pick_band_t(int lpr, bool two, int task) {
  switch (lpr) {
    case 1: return two ? solve_fn<BandEngine<2, 1, T>>(task) : solve_fn<BandEngine<1, 1, T>>(task);
    case 2: return two ? solve_fn<BandEngine<2, 2, T>>(task) : solve_fn<BandEngine<1, 2, T>>(task);
    case 4: return two ? solve_fn<BandEngine<2, 4, T>>(task) : solve_fn<BandEngine<1, 4, T>>(task);
    case 8: return two ? solve_fn<BandEngine<2, 8, T>>(task) : solve_fn<BandEngine<1, 8, T>>(task);
    case 16:
      return two ? solve_fn<BandEngine<2, 16, T>>(task) : solve_fn<BandEngine<1, 16, T>>(task);
    default: return nullptr;
  }
}

SolveFn pick_band_lp(const KParams& p, int units_per_wave_hint) {
  int lpr = 1;
  while (lpr * 4 < p.ell_k) lpr <<= 1;
  const bool two = units_per_wave_hint >= 2;
  if (p.vdtype == kBF16) return pick_band_t<ValBF16>(lpr, two, p.task);
  if (p.vdtype == kFP8) return pick_band_t<ValFP8>(lpr, two, p.task);
  return nullptr;
}

}  // namespace mbdp
