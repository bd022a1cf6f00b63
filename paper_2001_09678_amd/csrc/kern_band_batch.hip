// Banded scans from the census: batched launches (fixed-length bands).
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_band_batch(const Batch<ScanArgs>& b, int units, int LPL, int tau, int wpb, hipStream_t s) {
  shapes::band_batch_part<SRC_CENSUS>(b, units, LPL, tau, wpb, s);
}

}  // namespace mpvl
