// Full-range scans of a layered merge's later layers (the merge of the previous layer's
// two partial volumes as the data term): single-descriptor launches.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_layered(const ScanArgs& a, int src, int LPL, int K, bool banded, int wpb,
                       hipStream_t s) {
  if (src == SRC_CENSUS_OCC) return scan_full_occ(a, LPL, K, banded, wpb, s);
  shapes::full_part<SRC_MERGE>(a, LPL, K, banded, wpb, s);
}

}  // namespace mpvl
