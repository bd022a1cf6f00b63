// Full-range scans of the layered path merge (single-descriptor launches): the later
// layers, whose data term is the merge of the previous layer's two partial volumes, and
// the first layer with the occlusion weight (census source).
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <int LPL, int K, int SRC, int TAU, bool BANDED>
void go(const ScanArgs& a, int wpb, hipStream_t s) {
  const int units = a.gprefix[a.ndir];
  hipLaunchKernelGGL((k_scan_full<LPL, K, SRC, OUT_PART, TAU, BANDED>),
                     dim3((units + wpb - 1) / wpb), dim3(64 * wpb), 0, s, a);
}

template <int SRC, int TAU, bool BANDED>
void layout(const ScanArgs& a, int LPL, int K, int wpb, hipStream_t s) {
  if (LPL == 16) {
    if (K == 1) go<16, 1, SRC, TAU, BANDED>(a, wpb, s); else go<16, 2, SRC, TAU, BANDED>(a, wpb, s);
  } else if (LPL == 32) {
    if (K == 1) go<32, 1, SRC, TAU, BANDED>(a, wpb, s); else go<32, 2, SRC, TAU, BANDED>(a, wpb, s);
  } else {
    if (K == 1) go<64, 1, SRC, TAU, BANDED>(a, wpb, s); else go<64, 2, SRC, TAU, BANDED>(a, wpb, s);
  }
}

template <int SRC>
void taus(const ScanArgs& a, int LPL, int K, bool banded, int wpb, hipStream_t s) {
  if (banded) return layout<SRC, 0, true>(a, LPL, K, wpb, s);
  switch (a.tau) {
    case 1: return layout<SRC, 1, false>(a, LPL, K, wpb, s);
    case 2: return layout<SRC, 2, false>(a, LPL, K, wpb, s);
    case 4: return layout<SRC, 4, false>(a, LPL, K, wpb, s);
    default: return layout<SRC, 0, false>(a, LPL, K, wpb, s);
  }
}
}  // namespace

void scan_full_layered(const ScanArgs& a, int src, int LPL, int K, bool banded, int wpb,
                       hipStream_t s) {
  if (src == SRC_CENSUS_OCC) return taus<SRC_CENSUS_OCC>(a, LPL, K, banded, wpb, s);
  return taus<SRC_MERGE>(a, LPL, K, banded, wpb, s);
}

}  // namespace mpvl
