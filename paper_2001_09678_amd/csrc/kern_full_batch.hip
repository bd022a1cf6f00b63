// Full-range scan kernels: batched launches over a descriptor table.
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <int LPL, int K, int TAU, bool BANDED>
void go(const Batch<ScanArgs>& b, int units, int wpb, hipStream_t s) {
  hipLaunchKernelGGL((k_scan_full_batch<LPL, K, SRC_CENSUS, OUT_PART, TAU, BANDED>),
                     dim3((units + wpb - 1) / wpb), dim3(64 * wpb), 0, s, b);
}

template <int TAU, bool BANDED>
void layout(const Batch<ScanArgs>& b, int units, int LPL, int K, int wpb, hipStream_t s) {
  if (LPL == 16) {
    if (K == 1) go<16, 1, TAU, BANDED>(b, units, wpb, s); else go<16, 2, TAU, BANDED>(b, units, wpb, s);
  } else if (LPL == 32) {
    if (K == 1) go<32, 1, TAU, BANDED>(b, units, wpb, s); else go<32, 2, TAU, BANDED>(b, units, wpb, s);
  } else {
    if (K == 1) go<64, 1, TAU, BANDED>(b, units, wpb, s); else go<64, 2, TAU, BANDED>(b, units, wpb, s);
  }
}
}  // namespace

void scan_full_batch(const Batch<ScanArgs>& b, int units, int LPL, int K, int tau, bool banded,
                     int wpb, hipStream_t s) {
  if (banded) return layout<0, true>(b, units, LPL, K, wpb, s);
  switch (tau) {
    case 1: return layout<1, false>(b, units, LPL, K, wpb, s);
    case 2: return layout<2, false>(b, units, LPL, K, wpb, s);
    case 4: return layout<4, false>(b, units, LPL, K, wpb, s);
    default: return layout<0, false>(b, units, LPL, K, wpb, s);
  }
}

}  // namespace mpvl
