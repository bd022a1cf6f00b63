// Full-range scans of a layered merge's first layer with the occlusion weight (census
// source): single-descriptor launches.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_occ(const ScanArgs& a, int LPL, int K, bool banded, int wpb, hipStream_t s) {
  shapes::full_part<SRC_CENSUS_OCC>(a, LPL, K, banded, wpb, s);
}

}  // namespace mpvl
