// Full-range scans with gradient-weighted transitions of a layered merge's later layers:
// single-descriptor launches.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_grad_merge(const ScanArgs& a, int LPL, int K, bool banded, int wpb, hipStream_t s) {
  shapes::full_part<SRC_MERGE | SRC_GRAD>(a, LPL, K, banded, wpb, s);
}

}  // namespace mpvl
