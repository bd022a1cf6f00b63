// The top pyramid level's full-range scan (census source, sum of the paths) with the finer
// levels' census tiles run as extra blocks of the same launch.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <int LPL, int K, int TAU>
void go(const ScanArgs& a, const CenPyr& cp, int cen0, int ncen, int wpb, hipStream_t s) {
  const int nscan = (a.gprefix[a.ndir] + wpb - 1) / wpb;
  hipLaunchKernelGGL((k_scan_full_cen<LPL, K, TAU>), dim3(nscan + 2 * ncen), dim3(64 * wpb), 0, s, a, cp,
                     nscan, cen0, ncen);
}

template <int TAU>
void layout(const ScanArgs& a, const CenPyr& cp, int cen0, int ncen, int LPL, int K, int wpb, hipStream_t s) {
  if (LPL == 16) {
    if (K == 1) go<16, 1, TAU>(a, cp, cen0, ncen, wpb, s); else go<16, 2, TAU>(a, cp, cen0, ncen, wpb, s);
  } else if (LPL == 32) {
    if (K == 1) go<32, 1, TAU>(a, cp, cen0, ncen, wpb, s); else go<32, 2, TAU>(a, cp, cen0, ncen, wpb, s);
  } else {
    if (K == 1) go<64, 1, TAU>(a, cp, cen0, ncen, wpb, s); else go<64, 2, TAU>(a, cp, cen0, ncen, wpb, s);
  }
}
}  // namespace

void scan_full_cen(const ScanArgs& a, const CenPyr& cp, int cen0, int ncen, int LPL, int K, int wpb,
                   hipStream_t s) {
  switch (a.tau) {
    case 1: return layout<1>(a, cp, cen0, ncen, LPL, K, wpb, s);
    case 2: return layout<2>(a, cp, cen0, ncen, LPL, K, wpb, s);
    case 4: return layout<4>(a, cp, cen0, ncen, LPL, K, wpb, s);
    default: return layout<0>(a, cp, cen0, ncen, LPL, K, wpb, s);
  }
}

}  // namespace mpvl
