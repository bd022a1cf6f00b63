// Full-range scans with gradient-weighted transitions (eq. EU), batched launches: the
// census source (sum of the paths, first layer of a layered merge). The occlusion-weight
// and merge sources are in kern_full_batch_grad_layered.hip.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_batch_grad(const Batch<ScanArgs>& b, int src, int units, int LPL, int K, int tau,
                          bool banded, int wpb, hipStream_t s) {
  if (src_base(src) != SRC_CENSUS) return scan_full_batch_grad_layered(b, src, units, LPL, K, tau, banded, wpb, s);
  shapes::full_batch_part<SRC_CENSUS | SRC_GRAD>(b, units, LPL, K, tau, banded, wpb, s);
}

}  // namespace mpvl
