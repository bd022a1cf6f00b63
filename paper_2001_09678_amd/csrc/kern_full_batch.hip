// Full-range scans from the census: batched launches over a descriptor table.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_batch(const Batch<ScanArgs>& b, int units, int LPL, int K, int tau, bool banded,
                     int wpb, hipStream_t s) {
  shapes::full_batch_part<SRC_CENSUS>(b, units, LPL, K, tau, banded, wpb, s);
}

}  // namespace mpvl
