// Banded scans from the census and of the unfused export: single-descriptor launches.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_band(const ScanArgs& a, int LPL, int src, int out, bool v, int wpb, hipStream_t s) {
  if (src == SRC_CENSUS && out == OUT_PART) return shapes::band_part<SRC_CENSUS>(a, LPL, v, wpb, s);
  if (src == SRC_COST && out == OUT_PART) return scan_band_cost(a, LPL, v, wpb, s);
  // export path: cost volume in, canonical sums out
  if (out == OUT_U16) return shapes::band_var<SRC_COST, OUT_U16, 0>(a, LPL, v, wpb, s);
  shapes::band_var<SRC_COST, OUT_I32, 0>(a, LPL, v, wpb, s);
}

}  // namespace mpvl
