// Full-range scans of a layered merge's later layers: batched launches.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_batch_layered(const Batch<ScanArgs>& b, int src, int units, int LPL, int K, int tau,
                             bool banded, int wpb, hipStream_t s) {
  if (src == SRC_CENSUS_OCC) return scan_full_batch_occ(b, units, LPL, K, tau, banded, wpb, s);
  shapes::full_batch_part<SRC_MERGE>(b, units, LPL, K, tau, banded, wpb, s);
}

}  // namespace mpvl
