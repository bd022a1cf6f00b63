// Full-range scans with gradient-weighted transitions (eq. EU) from the census (sum of the
// paths, first layer of a layered merge): single-descriptor launches. The occlusion-weight
// and merge sources have units of their own.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_grad(const ScanArgs& a, int src, int LPL, int K, bool banded, int wpb, hipStream_t s) {
  if (src_occ(src)) return scan_full_grad_occ(a, LPL, K, banded, wpb, s);
  if (src_merge(src)) return scan_full_grad_merge(a, LPL, K, banded, wpb, s);
  shapes::full_part<SRC_CENSUS | SRC_GRAD>(a, LPL, K, banded, wpb, s);
}

}  // namespace mpvl
