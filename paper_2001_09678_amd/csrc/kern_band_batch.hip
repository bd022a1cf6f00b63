// Banded scan kernels: batched launches over a descriptor table.
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <int LPL, int TAU, bool VAR>
void go(const Batch<ScanArgs>& b, int units, int wpb, hipStream_t s) {
  hipLaunchKernelGGL((k_scan_band_batch<LPL, SRC_CENSUS, OUT_PART, TAU, VAR>),
                     dim3((units + wpb - 1) / wpb), dim3(64 * wpb), 0, s, b);
}

template <int TAU, bool VAR>
void lanes(const Batch<ScanArgs>& b, int units, int LPL, int wpb, hipStream_t s) {
  if (LPL == 16) go<16, TAU, VAR>(b, units, wpb, s);
  else if (LPL == 32) go<32, TAU, VAR>(b, units, wpb, s);
  else go<64, TAU, VAR>(b, units, wpb, s);
}

template <int TAU>
void var(const Batch<ScanArgs>& b, int units, int LPL, bool v, int wpb, hipStream_t s) {
  if (v) lanes<TAU, true>(b, units, LPL, wpb, s);
  else lanes<TAU, false>(b, units, LPL, wpb, s);
}
}  // namespace

void scan_band_batch(const Batch<ScanArgs>& b, int units, int LPL, int tau, bool v, int wpb,
                     hipStream_t s) {
  switch (tau) {
    case 1: return var<1>(b, units, LPL, v, wpb, s);
    case 2: return var<2>(b, units, LPL, v, wpb, s);
    case 4: return var<4>(b, units, LPL, v, wpb, s);
    default: return var<0>(b, units, LPL, v, wpb, s);
  }
}

}  // namespace mpvl
