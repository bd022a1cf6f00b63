// Full-range scan kernels: single-descriptor launches (fused and export paths).
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
using namespace mpvk;

bool full_layout_ok(int LPL, int K) {
  return (LPL == 16 || LPL == 32 || LPL == 64) && (K == 1 || K == 2);
}

namespace {
template <int LPL, int K, int SRC, int OUT, int TAU, bool BANDED>
void go(const ScanArgs& a, int wpb, hipStream_t s) {
  const int units = a.gprefix[a.ndir];
  hipLaunchKernelGGL((k_scan_full<LPL, K, SRC, OUT, TAU, BANDED>), dim3((units + wpb - 1) / wpb),
                     dim3(64 * wpb), 0, s, a);
}

template <int SRC, int OUT, int TAU, bool BANDED>
void layout(const ScanArgs& a, int LPL, int K, int wpb, hipStream_t s) {
  if (LPL == 16) {
    if (K == 1) go<16, 1, SRC, OUT, TAU, BANDED>(a, wpb, s); else go<16, 2, SRC, OUT, TAU, BANDED>(a, wpb, s);
  } else if (LPL == 32) {
    if (K == 1) go<32, 1, SRC, OUT, TAU, BANDED>(a, wpb, s); else go<32, 2, SRC, OUT, TAU, BANDED>(a, wpb, s);
  } else {
    if (K == 1) go<64, 1, SRC, OUT, TAU, BANDED>(a, wpb, s); else go<64, 2, SRC, OUT, TAU, BANDED>(a, wpb, s);
  }
}
}  // namespace

void scan_full(const ScanArgs& a, int LPL, int K, int src, int out, bool banded, int wpb,
               hipStream_t s) {
  if (src == SRC_CENSUS && out == OUT_PART) {
    if (banded) return layout<SRC_CENSUS, OUT_PART, 0, true>(a, LPL, K, wpb, s);
    switch (a.tau) {
      case 1: return layout<SRC_CENSUS, OUT_PART, 1, false>(a, LPL, K, wpb, s);
      case 2: return layout<SRC_CENSUS, OUT_PART, 2, false>(a, LPL, K, wpb, s);
      case 4: return layout<SRC_CENSUS, OUT_PART, 4, false>(a, LPL, K, wpb, s);
      default: return layout<SRC_CENSUS, OUT_PART, 0, false>(a, LPL, K, wpb, s);
    }
  }
  // export path: cost volume in, canonical sums out
  if (out == OUT_U16) {
    if (banded) return layout<SRC_COST, OUT_U16, 0, true>(a, LPL, K, wpb, s);
    return layout<SRC_COST, OUT_U16, 0, false>(a, LPL, K, wpb, s);
  }
  if (banded) return layout<SRC_COST, OUT_I32, 0, true>(a, LPL, K, wpb, s);
  return layout<SRC_COST, OUT_I32, 0, false>(a, LPL, K, wpb, s);
}

}  // namespace mpvl
