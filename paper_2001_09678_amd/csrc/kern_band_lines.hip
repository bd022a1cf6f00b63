// Batched banded scans with one line per lane for the directions that cross image rows.
#include "launch.hpp"
#include "lines.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
template <typename F>
bool with_shape(int cap, int tau, F&& f) {
  auto caps = [&](auto tc) {
    if (cap == 5) return f(std::integral_constant<int, 5>{}, tc), true;
    if (cap == 9) return f(std::integral_constant<int, 9>{}, tc), true;
    return false;
  };
  switch (tau) {
    case 1: return caps(std::integral_constant<int, 1>{});
    case 2: return caps(std::integral_constant<int, 2>{});
    case 4: return caps(std::integral_constant<int, 4>{});
    default: return false;
  }
}
}  // namespace

bool band_line_ok(int cap, int tau) {
  return with_shape(cap, tau, [](auto, auto) {}) && cap + 2 * (tau - 1) < 16 && cap <= 12;
}

void scan_lane_batch(const Batch<ScanArgs>& b, int units, int cap, int tau, bool p6, int wpb,
                     hipStream_t s) {
  with_shape(cap, tau, [&](auto cc, auto tc) {
    constexpr int CAP = decltype(cc)::value, TAU = decltype(tc)::value;
    const dim3 grid((units + wpb - 1) / wpb), block(64 * wpb);
    if (p6)
      hipLaunchKernelGGL((k_scan_lane_batch<TAU, CAP, true>), grid, block, 0, s, b);
    else
      hipLaunchKernelGGL((k_scan_lane_batch<TAU, CAP, false>), grid, block, 0, s, b);
  });
}

}  // namespace mpvl
