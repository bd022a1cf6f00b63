// Banded scans with gradient-weighted transitions (eq. EU) from the census, with or without
// the occlusion weight: single-descriptor launches. The merge source has a unit of its own.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_band_grad(const ScanArgs& a, int src, int LPL, bool v, int wpb, hipStream_t s) {
  if (src_merge(src)) return scan_band_grad_merge(a, LPL, v, wpb, s);
  if (src_occ(src)) return shapes::band_part<SRC_CENSUS_OCC | SRC_GRAD>(a, LPL, v, wpb, s);
  shapes::band_part<SRC_CENSUS | SRC_GRAD>(a, LPL, v, wpb, s);
}

}  // namespace mpvl
