// Banded scans of a layered merge: batched launches (fixed-length bands).
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_band_batch_layered(const Batch<ScanArgs>& b, int src, int units, int LPL, int tau, int wpb,
                             hipStream_t s) {
  if (src == SRC_CENSUS_OCC) return shapes::band_batch_part<SRC_CENSUS_OCC>(b, units, LPL, tau, wpb, s);
  shapes::band_batch_part<SRC_MERGE>(b, units, LPL, tau, wpb, s);
}

}  // namespace mpvl
