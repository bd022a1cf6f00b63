// The top pyramid level's full-range scan from the census (sum of the paths, or a layered
// merge's first layer with or without the occlusion weight) with the finer levels' census
// tiles run as extra blocks of the same launch. Gradient-weighted variants are in
// kern_full_cen_grad.hip.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <int LPL, int K, int SRC, int TAU>
void go(const ScanArgs& a, const CenPyr& cp, int cen0, int ncen, int wpb, hipStream_t s) {
  const int nscan = (a.gprefix[a.ndir] + wpb - 1) / wpb;
  hipLaunchKernelGGL((k_scan_full_cen<LPL, K, SRC, TAU>), dim3(nscan + 2 * ncen), dim3(64 * wpb), 0, s, a,
                     cp, nscan, cen0, ncen);
}

template <int SRC, int TAU>
void layout(const ScanArgs& a, const CenPyr& cp, int cen0, int ncen, int LPL, int K, int wpb, hipStream_t s) {
  if (LPL == 16) {
    if (K == 1) go<16, 1, SRC, TAU>(a, cp, cen0, ncen, wpb, s); else go<16, 2, SRC, TAU>(a, cp, cen0, ncen, wpb, s);
  } else if (LPL == 32) {
    if (K == 1) go<32, 1, SRC, TAU>(a, cp, cen0, ncen, wpb, s); else go<32, 2, SRC, TAU>(a, cp, cen0, ncen, wpb, s);
  } else {
    if (K == 1) go<64, 1, SRC, TAU>(a, cp, cen0, ncen, wpb, s); else go<64, 2, SRC, TAU>(a, cp, cen0, ncen, wpb, s);
  }
}

template <int SRC>
void taus(const ScanArgs& a, const CenPyr& cp, int cen0, int ncen, int LPL, int K, int wpb, hipStream_t s) {
  switch (a.tau) {
    case 1: return layout<SRC, 1>(a, cp, cen0, ncen, LPL, K, wpb, s);
    case 2: return layout<SRC, 2>(a, cp, cen0, ncen, LPL, K, wpb, s);
    case 4: return layout<SRC, 4>(a, cp, cen0, ncen, LPL, K, wpb, s);
    default: return layout<SRC, 0>(a, cp, cen0, ncen, LPL, K, wpb, s);
  }
}
}  // namespace

void scan_full_cen(const ScanArgs& a, int src, const CenPyr& cp, int cen0, int ncen, int LPL, int K,
                   int wpb, hipStream_t s) {
  if (src_grad(src)) return scan_full_cen_grad(a, src, cp, cen0, ncen, LPL, K, wpb, s);
  if (src_occ(src)) return taus<SRC_CENSUS_OCC>(a, cp, cen0, ncen, LPL, K, wpb, s);
  taus<SRC_CENSUS>(a, cp, cen0, ncen, LPL, K, wpb, s);
}

}  // namespace mpvl
