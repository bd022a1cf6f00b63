// Full-range scans of a layered merge's first layer with the occlusion weight: batched
// launches.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_batch_occ(const Batch<ScanArgs>& b, int units, int LPL, int K, int tau, bool banded,
                         int wpb, hipStream_t s) {
  shapes::full_batch_part<SRC_CENSUS_OCC>(b, units, LPL, K, tau, banded, wpb, s);
}

}  // namespace mpvl
