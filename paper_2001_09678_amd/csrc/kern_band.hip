// Banded scan kernels: single-descriptor launches (fused and export paths).
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <int LPL, int SRC, int OUT, int TAU, bool VAR>
void go(const ScanArgs& a, int wpb, hipStream_t s) {
  const int units = a.gprefix[a.ndir];
  hipLaunchKernelGGL((k_scan_band<LPL, SRC, OUT, TAU, VAR>), dim3((units + wpb - 1) / wpb),
                     dim3(64 * wpb), 0, s, a);
}

template <int SRC, int OUT, int TAU, bool VAR>
void lanes(const ScanArgs& a, int LPL, int wpb, hipStream_t s) {
  if (LPL == 16) go<16, SRC, OUT, TAU, VAR>(a, wpb, s);
  else if (LPL == 32) go<32, SRC, OUT, TAU, VAR>(a, wpb, s);
  else go<64, SRC, OUT, TAU, VAR>(a, wpb, s);
}

template <int SRC, int OUT, int TAU>
void var(const ScanArgs& a, int LPL, bool v, int wpb, hipStream_t s) {
  if (v) lanes<SRC, OUT, TAU, true>(a, LPL, wpb, s);
  else lanes<SRC, OUT, TAU, false>(a, LPL, wpb, s);
}
}  // namespace

void scan_band(const ScanArgs& a, int LPL, int src, int out, bool v, int wpb, hipStream_t s) {
  if (src == SRC_CENSUS && out == OUT_PART) {
    switch (a.tau) {
      case 1: return var<SRC_CENSUS, OUT_PART, 1>(a, LPL, v, wpb, s);
      case 2: return var<SRC_CENSUS, OUT_PART, 2>(a, LPL, v, wpb, s);
      case 4: return var<SRC_CENSUS, OUT_PART, 4>(a, LPL, v, wpb, s);
      default: return var<SRC_CENSUS, OUT_PART, 0>(a, LPL, v, wpb, s);
    }
  }
  if (out == OUT_U16) return var<SRC_COST, OUT_U16, 0>(a, LPL, v, wpb, s);
  return var<SRC_COST, OUT_I32, 0>(a, LPL, v, wpb, s);
}

}  // namespace mpvl
