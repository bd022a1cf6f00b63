// Banded scans of the layered path merge, batched launches over a descriptor table:
// later layers (merge of the previous layer's partials) and the first layer with the
// occlusion weight. Batches use fixed-length bands.
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <int LPL, int SRC, int TAU>
void go(const Batch<ScanArgs>& b, int units, int wpb, hipStream_t s) {
  hipLaunchKernelGGL((k_scan_band_batch<LPL, SRC, OUT_PART, TAU, false>),
                     dim3((units + wpb - 1) / wpb), dim3(64 * wpb), 0, s, b);
}

template <int SRC, int TAU>
void lanes(const Batch<ScanArgs>& b, int units, int LPL, int wpb, hipStream_t s) {
  if (LPL == 16) go<16, SRC, TAU>(b, units, wpb, s);
  else if (LPL == 32) go<32, SRC, TAU>(b, units, wpb, s);
  else go<64, SRC, TAU>(b, units, wpb, s);
}

template <int SRC>
void taus(const Batch<ScanArgs>& b, int units, int LPL, int tau, int wpb, hipStream_t s) {
  switch (tau) {
    case 1: return lanes<SRC, 1>(b, units, LPL, wpb, s);
    case 2: return lanes<SRC, 2>(b, units, LPL, wpb, s);
    case 4: return lanes<SRC, 4>(b, units, LPL, wpb, s);
    default: return lanes<SRC, 0>(b, units, LPL, wpb, s);
  }
}
}  // namespace

void scan_band_batch_layered(const Batch<ScanArgs>& b, int src, int units, int LPL, int tau, int wpb,
                             hipStream_t s) {
  if (src == SRC_CENSUS_OCC) return taus<SRC_CENSUS_OCC>(b, units, LPL, tau, wpb, s);
  return taus<SRC_MERGE>(b, units, LPL, tau, wpb, s);
}

}  // namespace mpvl
