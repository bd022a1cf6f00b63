// Banded scans of a layered merge: the later layers (merge of the previous layer's two
// partial volumes) and the first layer with the occlusion weight (single-descriptor
// launches).
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_band_layered(const ScanArgs& a, int src, int LPL, bool v, int wpb, hipStream_t s) {
  if (src == SRC_CENSUS_OCC) return shapes::band_part<SRC_CENSUS_OCC>(a, LPL, v, wpb, s);
  shapes::band_part<SRC_MERGE>(a, LPL, v, wpb, s);
}

}  // namespace mpvl
