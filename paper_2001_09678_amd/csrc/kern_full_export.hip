// Full-range scans of the unfused export: cost volume in, canonical (unnormalised) path
// energies out.
#include "scan_launch.hpp"

namespace mpvl {
using namespace mpvk;

void scan_full_export(const ScanArgs& a, int LPL, int K, int out, bool banded, int wpb, hipStream_t s) {
  if (out == OUT_U16) {
    if (banded) return shapes::full_layout<SRC_COST, OUT_U16, 0, true>(a, LPL, K, wpb, s);
    return shapes::full_layout<SRC_COST, OUT_U16, 0, false>(a, LPL, K, wpb, s);
  }
  if (banded) return shapes::full_layout<SRC_COST, OUT_I32, 0, true>(a, LPL, K, wpb, s);
  return shapes::full_layout<SRC_COST, OUT_I32, 0, false>(a, LPL, K, wpb, s);
}

}  // namespace mpvl
