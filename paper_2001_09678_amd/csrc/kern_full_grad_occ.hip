// Full-range scans with gradient-weighted transitions and the occlusion weight (first
// layer of a layered merge): single-descriptor launches.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_grad_occ(const ScanArgs& a, int LPL, int K, bool banded, int wpb, hipStream_t s) {
  shapes::full_part<SRC_CENSUS_OCC | SRC_GRAD>(a, LPL, K, banded, wpb, s);
}

}  // namespace mpvl
