// Banded scans with gradient-weighted transitions (eq. EU), batched launches (fixed-length
// bands): census, occlusion-weight and merge sources.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_band_batch_grad(const Batch<ScanArgs>& b, int src, int units, int LPL, int tau, int wpb,
                          hipStream_t s) {
  if (src_occ(src)) return shapes::band_batch_part<SRC_CENSUS_OCC | SRC_GRAD>(b, units, LPL, tau, wpb, s);
  if (src_merge(src)) return shapes::band_batch_part<SRC_MERGE | SRC_GRAD>(b, units, LPL, tau, wpb, s);
  shapes::band_batch_part<SRC_CENSUS | SRC_GRAD>(b, units, LPL, tau, wpb, s);
}

}  // namespace mpvl
