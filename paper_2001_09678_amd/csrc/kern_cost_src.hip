// Scans whose data term is a uint8 cost volume (the SSIM cost of the fused path), partial
// output: single-descriptor launches, full range and banded.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_cost(const ScanArgs& a, int LPL, int K, bool banded, int wpb, hipStream_t s) {
  shapes::full_part<SRC_COST>(a, LPL, K, banded, wpb, s);
}

void scan_band_cost(const ScanArgs& a, int LPL, bool var, int wpb, hipStream_t s) {
  shapes::band_part<SRC_COST>(a, LPL, var, wpb, s);
}

}  // namespace mpvl
