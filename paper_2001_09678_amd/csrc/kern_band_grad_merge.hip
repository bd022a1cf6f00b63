// Banded scans with gradient-weighted transitions of a layered merge's later layers:
// single-descriptor launches.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_band_grad_merge(const ScanArgs& a, int LPL, bool v, int wpb, hipStream_t s) {
  shapes::band_part<SRC_MERGE | SRC_GRAD>(a, LPL, v, wpb, s);
}

}  // namespace mpvl
