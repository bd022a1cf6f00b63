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
  return with_shape(cap, tau, [](auto, auto) {}) && cap + 2 * (tau - 1) <= 16 && cap <= 12;
}

void scan_lane_batch(const Batch<ScanArgs>& b, int units, int cap, int tau, int wpb, hipStream_t s) {
  with_shape(cap, tau, [&](auto cc, auto tc) {
    constexpr int CAP = decltype(cc)::value, TAU = decltype(tc)::value;
    hipLaunchKernelGGL((k_scan_lane_batch<TAU, CAP>), dim3((units + wpb - 1) / wpb), dim3(64 * wpb), 0, s, b);
  });
}

}  // namespace mpvl
