// Launch shapes of the scan kernels. Every kern_*.hip translation unit instantiates the
// kernels of one scan source through these templates (one source per unit keeps the
// units small enough to compile in parallel).
#pragma once
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
namespace shapes {
using namespace mpvk;

// ---- full-range scans, one descriptor
template <int LPL, int K, int SRC, int OUT, int TAU, bool BANDED>
inline void full_go(const ScanArgs& a, int wpb, hipStream_t s) {
  const int units = a.gprefix[a.ndir];
  hipLaunchKernelGGL((k_scan_full<LPL, K, SRC, OUT, TAU, BANDED>), dim3((units + wpb - 1) / wpb),
                     dim3(64 * wpb), 0, s, a);
}

template <int SRC, int OUT, int TAU, bool BANDED>
inline void full_layout(const ScanArgs& a, int LPL, int K, int wpb, hipStream_t s) {
  if (LPL == 16) {
    if (K == 1) full_go<16, 1, SRC, OUT, TAU, BANDED>(a, wpb, s); else full_go<16, 2, SRC, OUT, TAU, BANDED>(a, wpb, s);
  } else if (LPL == 32) {
    if (K == 1) full_go<32, 1, SRC, OUT, TAU, BANDED>(a, wpb, s); else full_go<32, 2, SRC, OUT, TAU, BANDED>(a, wpb, s);
  } else {
    if (K == 1) full_go<64, 1, SRC, OUT, TAU, BANDED>(a, wpb, s); else full_go<64, 2, SRC, OUT, TAU, BANDED>(a, wpb, s);
  }
}

// Partial output: compile-time tau 1, 2, 4, runtime tau otherwise and for band masks.
template <int SRC>
inline void full_part(const ScanArgs& a, int LPL, int K, bool banded, int wpb, hipStream_t s) {
  if (banded) return full_layout<SRC, OUT_PART, 0, true>(a, LPL, K, wpb, s);
  switch (a.tau) {
    case 1: return full_layout<SRC, OUT_PART, 1, false>(a, LPL, K, wpb, s);
    case 2: return full_layout<SRC, OUT_PART, 2, false>(a, LPL, K, wpb, s);
    case 4: return full_layout<SRC, OUT_PART, 4, false>(a, LPL, K, wpb, s);
    default: return full_layout<SRC, OUT_PART, 0, false>(a, LPL, K, wpb, s);
  }
}

// ---- full-range scans, batched over a descriptor table
template <int LPL, int K, int SRC, int TAU, bool BANDED>
inline void full_batch_go(const Batch<ScanArgs>& b, int units, int wpb, hipStream_t s) {
  hipLaunchKernelGGL((k_scan_full_batch<LPL, K, SRC, OUT_PART, TAU, BANDED>),
                     dim3((units + wpb - 1) / wpb), dim3(64 * wpb), 0, s, b);
}

template <int SRC, int TAU, bool BANDED>
inline void full_batch_layout(const Batch<ScanArgs>& b, int units, int LPL, int K, int wpb, hipStream_t s) {
  if (LPL == 16) {
    if (K == 1) full_batch_go<16, 1, SRC, TAU, BANDED>(b, units, wpb, s); else full_batch_go<16, 2, SRC, TAU, BANDED>(b, units, wpb, s);
  } else if (LPL == 32) {
    if (K == 1) full_batch_go<32, 1, SRC, TAU, BANDED>(b, units, wpb, s); else full_batch_go<32, 2, SRC, TAU, BANDED>(b, units, wpb, s);
  } else {
    if (K == 1) full_batch_go<64, 1, SRC, TAU, BANDED>(b, units, wpb, s); else full_batch_go<64, 2, SRC, TAU, BANDED>(b, units, wpb, s);
  }
}

template <int SRC>
inline void full_batch_part(const Batch<ScanArgs>& b, int units, int LPL, int K, int tau, bool banded,
                            int wpb, hipStream_t s) {
  if (banded) return full_batch_layout<SRC, 0, true>(b, units, LPL, K, wpb, s);
  switch (tau) {
    case 1: return full_batch_layout<SRC, 1, false>(b, units, LPL, K, wpb, s);
    case 2: return full_batch_layout<SRC, 2, false>(b, units, LPL, K, wpb, s);
    case 4: return full_batch_layout<SRC, 4, false>(b, units, LPL, K, wpb, s);
    default: return full_batch_layout<SRC, 0, false>(b, units, LPL, K, wpb, s);
  }
}

// ---- banded scans, one descriptor
template <int LPL, int SRC, int OUT, int TAU, bool VAR>
inline void band_go(const ScanArgs& a, int wpb, hipStream_t s) {
  const int units = a.gprefix[a.ndir];
  hipLaunchKernelGGL((k_scan_band<LPL, SRC, OUT, TAU, VAR>), dim3((units + wpb - 1) / wpb),
                     dim3(64 * wpb), 0, s, a);
}

template <int SRC, int OUT, int TAU>
inline void band_var(const ScanArgs& a, int LPL, bool v, int wpb, hipStream_t s) {
  if (LPL == 16) {
    if (v) band_go<16, SRC, OUT, TAU, true>(a, wpb, s); else band_go<16, SRC, OUT, TAU, false>(a, wpb, s);
  } else if (LPL == 32) {
    if (v) band_go<32, SRC, OUT, TAU, true>(a, wpb, s); else band_go<32, SRC, OUT, TAU, false>(a, wpb, s);
  } else {
    if (v) band_go<64, SRC, OUT, TAU, true>(a, wpb, s); else band_go<64, SRC, OUT, TAU, false>(a, wpb, s);
  }
}

template <int SRC>
inline void band_part(const ScanArgs& a, int LPL, bool v, int wpb, hipStream_t s) {
  switch (a.tau) {
    case 1: return band_var<SRC, OUT_PART, 1>(a, LPL, v, wpb, s);
    case 2: return band_var<SRC, OUT_PART, 2>(a, LPL, v, wpb, s);
    case 4: return band_var<SRC, OUT_PART, 4>(a, LPL, v, wpb, s);
    default: return band_var<SRC, OUT_PART, 0>(a, LPL, v, wpb, s);
  }
}

// ---- banded scans, batched (batches use fixed-length bands)
template <int LPL, int SRC, int TAU>
inline void band_batch_go(const Batch<ScanArgs>& b, int units, int wpb, hipStream_t s) {
  hipLaunchKernelGGL((k_scan_band_batch<LPL, SRC, OUT_PART, TAU, false>), dim3((units + wpb - 1) / wpb),
                     dim3(64 * wpb), 0, s, b);
}

template <int SRC>
inline void band_batch_part(const Batch<ScanArgs>& b, int units, int LPL, int tau, int wpb, hipStream_t s) {
  auto lanes = [&](auto tc) {
    constexpr int TAU = decltype(tc)::value;
    if (LPL == 16) band_batch_go<16, SRC, TAU>(b, units, wpb, s);
    else if (LPL == 32) band_batch_go<32, SRC, TAU>(b, units, wpb, s);
    else band_batch_go<64, SRC, TAU>(b, units, wpb, s);
  };
  switch (tau) {
    case 1: return lanes(std::integral_constant<int, 1>{});
    case 2: return lanes(std::integral_constant<int, 2>{});
    case 4: return lanes(std::integral_constant<int, 4>{});
    default: return lanes(std::integral_constant<int, 0>{});
  }
}

}  // namespace shapes
}  // namespace mpvl
