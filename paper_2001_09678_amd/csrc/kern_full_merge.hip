// Full-range scans of the layered path merge's later layers: the data term is the merge
// of the previous layer's two partial volumes (single-descriptor launches).
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <int LPL, int K, int TAU, bool BANDED>
void go(const ScanArgs& a, int wpb, hipStream_t s) {
  const int units = a.gprefix[a.ndir];
  hipLaunchKernelGGL((k_scan_full<LPL, K, SRC_MERGE, OUT_PART, TAU, BANDED>),
                     dim3((units + wpb - 1) / wpb), dim3(64 * wpb), 0, s, a);
}

template <int TAU, bool BANDED>
void layout(const ScanArgs& a, int LPL, int K, int wpb, hipStream_t s) {
  if (LPL == 16) {
    if (K == 1) go<16, 1, TAU, BANDED>(a, wpb, s); else go<16, 2, TAU, BANDED>(a, wpb, s);
  } else if (LPL == 32) {
    if (K == 1) go<32, 1, TAU, BANDED>(a, wpb, s); else go<32, 2, TAU, BANDED>(a, wpb, s);
  } else {
    if (K == 1) go<64, 1, TAU, BANDED>(a, wpb, s); else go<64, 2, TAU, BANDED>(a, wpb, s);
  }
}
}  // namespace

void scan_full_merge(const ScanArgs& a, int LPL, int K, bool banded, int wpb, hipStream_t s) {
  if (banded) return layout<0, true>(a, LPL, K, wpb, s);
  switch (a.tau) {
    case 1: return layout<1, false>(a, LPL, K, wpb, s);
    case 2: return layout<2, false>(a, LPL, K, wpb, s);
    case 4: return layout<4, false>(a, LPL, K, wpb, s);
    default: return layout<0, false>(a, LPL, K, wpb, s);
  }
}

}  // namespace mpvl
