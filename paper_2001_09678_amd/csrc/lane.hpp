// Cross-lane building blocks for gfx950 (CDNA4, wave64).
//
// A Viterbi line is mapped to a group of LPL consecutive lanes (LPL = 16, 32 or 64), so
// a wave carries 64/LPL lines. Neighbour exchange along the disparity axis is a lane
// shift inside the group: DPP row/wave shifts, with lanes that would read outside the
// group receiving a fill value. Group-wide minima use a rotate butterfly inside each
// 16-lane row (DPP row_ror 8/4/2/1) and then the gfx950 permlane16/permlane32 swaps to
// combine rows, which leaves the minimum in every lane of the group.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpvk {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// "Absent node" value of the 16-bit packed energies. Real normalised energies stay
// below 24 + lambda*tau <= 4024 and an absent node never grows past INF16 + 3*4024,
// so packed adds never wrap.
constexpr uint32_t INF16 = 0x3FFFu;
constexpr uint32_t INF2 = 0x3FFF3FFFu;
constexpr uint32_t INF32 = 0x3FFFFFFFu;

__device__ __forceinline__ uint32_t pk_min(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t pk_max(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t pk_add(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) + __builtin_bit_cast(u16x2, b));
}
__device__ __forceinline__ uint32_t pk_sub(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, a) - __builtin_bit_cast(u16x2, b));
}
typedef short i16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_max_i(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(i16x2, a),
                                                                __builtin_bit_cast(i16x2, b)));
}
__device__ __forceinline__ uint32_t pk_sub_i(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(i16x2, a) - __builtin_bit_cast(i16x2, b));
}
__device__ __forceinline__ uint32_t pk_add_i(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(i16x2, a) + __builtin_bit_cast(i16x2, b));
}
__device__ __forceinline__ int lo16s(uint32_t v) { return (int)(short)(v & 0xFFFFu); }
__device__ __forceinline__ int hi16s(uint32_t v) { return (int)v >> 16; }
__device__ __forceinline__ uint32_t splat16(uint32_t v) { return v | (v << 16); }
__device__ __forceinline__ uint32_t lo16(uint32_t v) { return v & 0xFFFFu; }
__device__ __forceinline__ uint32_t hi16(uint32_t v) { return v >> 16; }
// (hi << 16) | (lo >> 16): the upper half of `lo` moves down, the lower half of `hi` moves up
__device__ __forceinline__ uint32_t funnel16(uint32_t hi, uint32_t lo) {
  return __builtin_amdgcn_alignbit(hi, lo, 16);
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, 0xF, 0xF, false);
}

// DPP controls (GFX9 encoding)
constexpr int ROW_SHL1 = 0x101;
constexpr int ROW_SHR1 = 0x111;
constexpr int ROW_ROR1 = 0x121, ROW_ROR2 = 0x122, ROW_ROR4 = 0x124, ROW_ROR8 = 0x128;
constexpr int WAVE_SHL1 = 0x130;
constexpr int ROW_BCAST15 = 0x142, ROW_BCAST31 = 0x143;
constexpr int WAVE_SHR1 = 0x138;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Value of lane l-1 of the same group (fill for the group's first lane).
template <int LPL>
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v, uint32_t fill) {
  if constexpr (LPL == 16) {
    return dpp<ROW_SHR1>(fill, v);
  } else if constexpr (LPL == 64) {
    return dpp<WAVE_SHR1>(fill, v);
  } else {
    uint32_t t = dpp<WAVE_SHR1>(fill, v);
    return (lane_id() & 31) ? t : fill;
  }
}

// Value of lane l+1 of the same group (fill for the group's last lane).
template <int LPL>
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v, uint32_t fill) {
  if constexpr (LPL == 16) {
    return dpp<ROW_SHL1>(fill, v);
  } else if constexpr (LPL == 64) {
    return dpp<WAVE_SHL1>(fill, v);
  } else {
    uint32_t t = dpp<WAVE_SHL1>(fill, v);
    return ((lane_id() & 31) != 31) ? t : fill;
  }
}

// Value of lane l-n (n > 0: from below; n < 0: from above) of the same group, `fill`
// where that lane is outside the group. Generic path through ds_bpermute.
template <int LPL>
__device__ __forceinline__ uint32_t from_lane_offset(uint32_t v, int n, uint32_t fill) {
  const int lane = lane_id();
  const int l = lane % LPL;
  const int src = l - n;
  const int got = __builtin_amdgcn_ds_bpermute((lane - n) << 2, (int)v);
  return (src >= 0 && src < LPL) ? (uint32_t)got : fill;
}

// Lane shift by a small runtime amount inside 16-lane rows (DPP), any amount otherwise.
template <int LPL>
__device__ __forceinline__ uint32_t shift_up(uint32_t v, int n, uint32_t fill) {
  if constexpr (LPL == 16) {
    switch (n) {
      case 0: return v;
      case 1: return dpp<0x111>(fill, v);
      case 2: return dpp<0x112>(fill, v);
      case 3: return dpp<0x113>(fill, v);
      case 4: return dpp<0x114>(fill, v);
      case 5: return dpp<0x115>(fill, v);
      case 6: return dpp<0x116>(fill, v);
      case 7: return dpp<0x117>(fill, v);
      case 8: return dpp<0x118>(fill, v);
      default: return from_lane_offset<LPL>(v, n, fill);
    }
  } else {
    if (n == 0) return v;
    if (n == 1) return from_prev_lane<LPL>(v, fill);
    return from_lane_offset<LPL>(v, n, fill);
  }
}

template <int LPL>
__device__ __forceinline__ uint32_t shift_down(uint32_t v, int n, uint32_t fill) {
  if constexpr (LPL == 16) {
    switch (n) {
      case 0: return v;
      case 1: return dpp<0x101>(fill, v);
      case 2: return dpp<0x102>(fill, v);
      case 3: return dpp<0x103>(fill, v);
      case 4: return dpp<0x104>(fill, v);
      case 5: return dpp<0x105>(fill, v);
      case 6: return dpp<0x106>(fill, v);
      case 7: return dpp<0x107>(fill, v);
      case 8: return dpp<0x108>(fill, v);
      default: return from_lane_offset<LPL>(v, -n, fill);
    }
  } else {
    if (n == 0) return v;
    if (n == 1) return from_next_lane<LPL>(v, fill);
    return from_lane_offset<LPL>(v, -n, fill);
  }
}

// Compile-time lane shifts: value of lane l-N (up) / l+N (down) of the same group.
template <int LPL, int N>
__device__ __forceinline__ uint32_t shift_up_c(uint32_t v, uint32_t fill) {
  if constexpr (N == 0)
    return v;
  else if constexpr (LPL == 16)
    return dpp<0x110 + N>(fill, v);  // row_shr:N
  else if constexpr (N == 1)
    return from_prev_lane<LPL>(v, fill);
  else
    return from_lane_offset<LPL>(v, N, fill);
}

template <int LPL, int N>
__device__ __forceinline__ uint32_t shift_down_c(uint32_t v, uint32_t fill) {
  if constexpr (N == 0)
    return v;
  else if constexpr (LPL == 16)
    return dpp<0x100 + N>(fill, v);  // row_shl:N
  else if constexpr (N == 1)
    return from_next_lane<LPL>(v, fill);
  else
    return from_lane_offset<LPL>(v, -N, fill);
}

constexpr int ceil_log2(int v) { return v <= 1 ? 0 : 1 + ceil_log2((v + 1) / 2); }

// Minimum over the LPL lanes of a group, returned in every lane of the group.
template <int LPL>
__device__ __forceinline__ uint32_t group_min(uint32_t v) {
  v = min(v, dpp<ROW_ROR8>(v, v));
  v = min(v, dpp<ROW_ROR4>(v, v));
  v = min(v, dpp<ROW_ROR2>(v, v));
  v = min(v, dpp<ROW_ROR1>(v, v));
  if constexpr (LPL >= 32) {
    auto s = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = min((uint32_t)s[0], (uint32_t)s[1]);
  }
  if constexpr (LPL >= 64) {
    auto s = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    v = min((uint32_t)s[0], (uint32_t)s[1]);
  }
  return v;
}

// ---- complement-encoded energies: u = INF - value, absent node = 0, best = largest.
// DPP shifts fill with 0 (hardware bound_ctrl), i.e. with "absent".
template <int CTRL>
__device__ __forceinline__ int dpp0(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

// Value of lane l-N (up) / l+N (down) of the same group, 0 outside the group.
template <int LPL, int N>
__device__ __forceinline__ int zshift_up(int v) {
  if constexpr (N == 0) {
    return v;
  } else if constexpr (LPL == 16) {
    return dpp0<0x110 + N>(v);  // row_shr:N
  } else if constexpr (N == 1 && LPL == 64) {
    return dpp0<WAVE_SHR1>(v);
  } else if constexpr (N == 1) {
    const int t = dpp0<WAVE_SHR1>(v);
    return (lane_id() & 31) ? t : 0;
  } else {
    const int lane = lane_id();
    const int src = lane % LPL - N;
    const int got = __builtin_amdgcn_ds_bpermute((lane - N) << 2, v);
    return src >= 0 ? got : 0;
  }
}

template <int LPL, int N>
__device__ __forceinline__ int zshift_down(int v) {
  if constexpr (N == 0) {
    return v;
  } else if constexpr (LPL == 16) {
    return dpp0<0x100 + N>(v);  // row_shl:N
  } else if constexpr (N == 1 && LPL == 64) {
    return dpp0<WAVE_SHL1>(v);
  } else if constexpr (N == 1) {
    const int t = dpp0<WAVE_SHL1>(v);
    return ((lane_id() & 31) != 31) ? t : 0;
  } else {
    const int lane = lane_id();
    const int src = lane % LPL + N;
    const int got = __builtin_amdgcn_ds_bpermute((lane + N) << 2, v);
    return src < LPL ? got : 0;
  }
}

// Maximum over the LPL lanes of a group (signed), in every lane of the group.
template <int LPL>
__device__ __forceinline__ int group_max(int v) {
  v = max(v, dpp0<ROW_ROR8>(v));
  v = max(v, dpp0<ROW_ROR4>(v));
  v = max(v, dpp0<ROW_ROR2>(v));
  v = max(v, dpp0<ROW_ROR1>(v));
  if constexpr (LPL >= 32) {
    auto s = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = max((int)s[0], (int)s[1]);
  }
  if constexpr (LPL >= 64) {
    auto s = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    v = max((int)s[0], (int)s[1]);
  }
  return v;
}

// Maximum over the whole wave, returned wave-uniform (scalar): a rotate butterfly inside
// each 16-lane row, then the four row maxima read into scalar registers.
__device__ __forceinline__ int wave_max_s(int v) {
  v = max(v, dpp0<ROW_ROR8>(v));
  v = max(v, dpp0<ROW_ROR4>(v));
  v = max(v, dpp0<ROW_ROR2>(v));
  v = max(v, dpp0<ROW_ROR1>(v));
  // rows 1 and 3 take the maximum of the row before; rows 2 and 3 that of lane 31
  // (disabled rows read INT_MIN, the identity of max, so the DPP fuses into the max)
  v = max(v, __builtin_amdgcn_update_dpp((int)0x80000000, v, ROW_BCAST15, 0xA, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp((int)0x80000000, v, ROW_BCAST31, 0xC, 0xF, false));
  return __builtin_amdgcn_readlane(v, 63);
}

// Cache policy of the partial-volume stores whose wave writes whole cache lines at a time
// (full-range scans, one line per lane): non-temporal. The volumes are written once, read
// once by the reduce after the whole scan, and (batched) far larger than the caches;
// streaming them past the caches leaves room for the census words that the scans reuse.
// The lane-group banded scan writes 16-byte pieces of many lines per step, which the L2 has
// to merge: those stores keep the default policy (measured: non-temporal is slower there).
constexpr int kPartStorePolicy = 2;  // nt

// Buffer resource over `p` (raw addressing, no stride; gfx9 data-format word): loads and
// stores then take a scalar offset plus a 32-bit lane offset, with no 64-bit address math.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t make_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, 0x7FFFFFFF, 0x00020000);
}
__device__ __forceinline__ uint32_t buf_ld32(rsrc_t r, uint32_t voff, uint32_t soff) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ uint32_t buf_ld16(rsrc_t r, uint32_t voff, uint32_t soff) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ uint32_t buf_ld8(rsrc_t r, uint32_t voff, uint32_t soff) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(r, (int)voff, (int)soff, 0);
}

// Minimum over aligned groups of N lanes (N = 1, 2, 4, 8, 16), in every lane of the group.
template <int N>
__device__ __forceinline__ uint32_t small_group_min(uint32_t v) {
  if constexpr (N >= 2) v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true));
  if constexpr (N >= 4) v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true));
  if constexpr (N >= 8) v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true));
  if constexpr (N >= 16) v = min(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true));
  return v;
}

}  // namespace mpvk
