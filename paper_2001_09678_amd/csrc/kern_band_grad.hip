// Banded scans with gradient-weighted transitions (eq. EU): the census source (sum of the
// paths, first layer of a layered merge, with or without the occlusion weight) and the
// merge source of the later layers (single-descriptor launches).
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <int LPL, int SRC, int TAU, bool VAR>
void go(const ScanArgs& a, int wpb, hipStream_t s) {
  const int units = a.gprefix[a.ndir];
  hipLaunchKernelGGL((k_scan_band<LPL, SRC, OUT_PART, TAU, VAR>),
                     dim3((units + wpb - 1) / wpb), dim3(64 * wpb), 0, s, a);
}

template <int SRC, int TAU, bool VAR>
void lanes(const ScanArgs& a, int LPL, int wpb, hipStream_t s) {
  if (LPL == 16) go<16, SRC, TAU, VAR>(a, wpb, s);
  else if (LPL == 32) go<32, SRC, TAU, VAR>(a, wpb, s);
  else go<64, SRC, TAU, VAR>(a, wpb, s);
}

template <int SRC, int TAU>
void var(const ScanArgs& a, int LPL, bool v, int wpb, hipStream_t s) {
  if (v) lanes<SRC, TAU, true>(a, LPL, wpb, s);
  else lanes<SRC, TAU, false>(a, LPL, wpb, s);
}

template <int SRC>
void taus(const ScanArgs& a, int LPL, bool v, int wpb, hipStream_t s) {
  switch (a.tau) {
    case 1: return var<SRC, 1>(a, LPL, v, wpb, s);
    case 2: return var<SRC, 2>(a, LPL, v, wpb, s);
    case 4: return var<SRC, 4>(a, LPL, v, wpb, s);
    default: return var<SRC, 0>(a, LPL, v, wpb, s);
  }
}
}  // namespace

void scan_band_grad(const ScanArgs& a, int src, int LPL, bool v, int wpb, hipStream_t s) {
  switch (src_base(src)) {
    case SRC_CENSUS_OCC: return taus<SRC_CENSUS_OCC | SRC_GRAD>(a, LPL, v, wpb, s);
    case SRC_MERGE: return taus<SRC_MERGE | SRC_GRAD>(a, LPL, v, wpb, s);
    default: return taus<SRC_CENSUS | SRC_GRAD>(a, LPL, v, wpb, s);
  }
}

}  // namespace mpvl
