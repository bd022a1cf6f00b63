// Full-range scans with gradient-weighted transitions (eq. EU): the census source (sum of
// the paths, first layer of a layered merge, with or without the occlusion weight) and the
// merge source of the later layers (single-descriptor launches).
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

void scan_full_grad(const ScanArgs& a, int src, int LPL, int K, bool banded, int wpb, hipStream_t s) {
  switch (src_base(src)) {
    case SRC_CENSUS_OCC: return taus<SRC_CENSUS_OCC | SRC_GRAD>(a, LPL, K, banded, wpb, s);
    case SRC_MERGE: return taus<SRC_MERGE | SRC_GRAD>(a, LPL, K, banded, wpb, s);
    default: return taus<SRC_CENSUS | SRC_GRAD>(a, LPL, K, banded, wpb, s);
  }
}

}  // namespace mpvl
