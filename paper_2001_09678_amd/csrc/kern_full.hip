// Full-range scans from the census (sum of the paths, first layer of a layered merge):
// single-descriptor launches.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

bool full_layout_ok(int LPL, int K) {
  return (LPL == 16 || LPL == 32 || LPL == 64) && (K == 1 || K == 2);
}

void scan_full(const ScanArgs& a, int LPL, int K, int src, int out, bool banded, int wpb,
               hipStream_t s) {
  if (src == SRC_CENSUS && out == OUT_PART) return shapes::full_part<SRC_CENSUS>(a, LPL, K, banded, wpb, s);
  if (src == SRC_COST && out == OUT_PART) return scan_full_cost(a, LPL, K, banded, wpb, s);
  scan_full_export(a, LPL, K, out, banded, wpb, s);
}

}  // namespace mpvl
