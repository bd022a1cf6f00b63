// Full-range scans of the layered path merge, batched launches over a descriptor table:
// later layers (merge of the previous layer's partials) and the first layer with the
// occlusion weight.
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <int LPL, int K, int SRC, int TAU, bool BANDED>
void go(const Batch<ScanArgs>& b, int units, int wpb, hipStream_t s) {
  hipLaunchKernelGGL((k_scan_full_batch<LPL, K, SRC, OUT_PART, TAU, BANDED>),
                     dim3((units + wpb - 1) / wpb), dim3(64 * wpb), 0, s, b);
}

template <int SRC, int TAU, bool BANDED>
void layout(const Batch<ScanArgs>& b, int units, int LPL, int K, int wpb, hipStream_t s) {
  if (LPL == 16) {
    if (K == 1) go<16, 1, SRC, TAU, BANDED>(b, units, wpb, s); else go<16, 2, SRC, TAU, BANDED>(b, units, wpb, s);
  } else if (LPL == 32) {
    if (K == 1) go<32, 1, SRC, TAU, BANDED>(b, units, wpb, s); else go<32, 2, SRC, TAU, BANDED>(b, units, wpb, s);
  } else {
    if (K == 1) go<64, 1, SRC, TAU, BANDED>(b, units, wpb, s); else go<64, 2, SRC, TAU, BANDED>(b, units, wpb, s);
  }
}

template <int SRC>
void taus(const Batch<ScanArgs>& b, int units, int LPL, int K, int tau, bool banded, int wpb,
          hipStream_t s) {
  if (banded) return layout<SRC, 0, true>(b, units, LPL, K, wpb, s);
  switch (tau) {
    case 1: return layout<SRC, 1, false>(b, units, LPL, K, wpb, s);
    case 2: return layout<SRC, 2, false>(b, units, LPL, K, wpb, s);
    case 4: return layout<SRC, 4, false>(b, units, LPL, K, wpb, s);
    default: return layout<SRC, 0, false>(b, units, LPL, K, wpb, s);
  }
}
}  // namespace

void scan_full_batch_layered(const Batch<ScanArgs>& b, int src, int units, int LPL, int K, int tau,
                             bool banded, int wpb, hipStream_t s) {
  if (src == SRC_CENSUS_OCC) return taus<SRC_CENSUS_OCC>(b, units, LPL, K, tau, banded, wpb, s);
  return taus<SRC_MERGE>(b, units, LPL, K, tau, banded, wpb, s);
}

}  // namespace mpvl
