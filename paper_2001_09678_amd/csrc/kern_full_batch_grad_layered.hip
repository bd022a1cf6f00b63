// Full-range scans with gradient-weighted transitions (eq. EU) of a layered merge, batched
// launches: the first layer with the occlusion weight and the later layers' merge source.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_batch_grad_layered(const Batch<ScanArgs>& b, int src, int units, int LPL, int K, int tau,
                                  bool banded, int wpb, hipStream_t s) {
  if (src_occ(src)) return shapes::full_batch_part<SRC_CENSUS_OCC | SRC_GRAD>(b, units, LPL, K, tau, banded, wpb, s);
  shapes::full_batch_part<SRC_MERGE | SRC_GRAD>(b, units, LPL, K, tau, banded, wpb, s);
}

}  // namespace mpvl
