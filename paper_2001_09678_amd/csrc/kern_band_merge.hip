// Banded scans of the layered path merge's later layers: the data term is the merge of
// the previous layer's two partial volumes (single-descriptor launches).
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <int LPL, int TAU, bool VAR>
void go(const ScanArgs& a, int wpb, hipStream_t s) {
  const int units = a.gprefix[a.ndir];
  hipLaunchKernelGGL((k_scan_band<LPL, SRC_MERGE, OUT_PART, TAU, VAR>),
                     dim3((units + wpb - 1) / wpb), dim3(64 * wpb), 0, s, a);
}

template <int TAU, bool VAR>
void lanes(const ScanArgs& a, int LPL, int wpb, hipStream_t s) {
  if (LPL == 16) go<16, TAU, VAR>(a, wpb, s);
  else if (LPL == 32) go<32, TAU, VAR>(a, wpb, s);
  else go<64, TAU, VAR>(a, wpb, s);
}

template <int TAU>
void var(const ScanArgs& a, int LPL, bool v, int wpb, hipStream_t s) {
  if (v) lanes<TAU, true>(a, LPL, wpb, s);
  else lanes<TAU, false>(a, LPL, wpb, s);
}
}  // namespace

void scan_band_merge(const ScanArgs& a, int LPL, bool v, int wpb, hipStream_t s) {
  switch (a.tau) {
    case 1: return var<1>(a, LPL, v, wpb, s);
    case 2: return var<2>(a, LPL, v, wpb, s);
    case 4: return var<4>(a, LPL, v, wpb, s);
    default: return var<0>(a, LPL, v, wpb, s);
  }
}

}  // namespace mpvl
