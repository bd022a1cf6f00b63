// HIP kernels of the MPV stereo matcher for gfx950.
//
// Data layout in HBM
//   images      uint8 [H][pitch]
//   census      uint32 [H][cpitch], pixel (x, y) at y*cpitch + cmargin + x; the left
//               margin keeps the cost loads of candidates x-d < 0 inside the buffer
//   partials    uint8 [P][H][W][capP]: one normalised energy volume per scan direction
//   bands       int16 lo [H][W], uint8 len [H][W]
//   disparity   int16 [H][W], -1 = invalid
//
// Scan kernels (the directed-path Viterbi of Section 3.2, eq. e(p,u)): one line of one
// direction per group of LPL lanes; a lane holds 2K disparities of the line as packed
// 16-bit energies (full range) or one disparity (band). The min over predecessors uses
// the decomposition of Section 3.3: the envelope of lambda*|d-d'| is built by sweeps
// along the disparity axis (here as doubling steps s = 1, 2, 4, ... so that a window of
// tau-1 neighbours takes log2(tau) cross-lane steps), and the truncation at tau is one
// more candidate, the previous minimum plus lambda*tau. Full-range scans keep their packed
// 16-bit energies normalised (previous minimum subtracted, so the candidate is lambda*tau);
// banded scans keep unnormalised 32-bit energies and take the candidate from the previous
// pixel's minimum, computed beside the next step instead of on its dependent chain. The
// stored partials are always the energy minus the pixel's minimum over its disparities.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <utility>
#include <type_traits>

#include "lane.hpp"
#include "types.hpp"

namespace mpvk {

// Band of pixel p, clamped so that any map stays in bounds: 0 <= b0 < D, 1 <= bn <= min(cap, D-b0).
__device__ __forceinline__ void band_at(const int16_t* lo, const uint8_t* len, size_t p, int D,
                                        int cap, int& b0, int& bn) {
  b0 = lo ? min(max((int)lo[p], 0), D - 1) : 0;
  bn = len ? (int)len[p] : cap;
  bn = min(max(bn, 1), min(cap, D - b0));
}

static __constant__ int c_dx[8] = {+1, -1, 0, 0, +1, -1, -1, +1};
static __constant__ int c_dy[8] = {0, 0, +1, -1, +1, -1, +1, -1};

// ---------------------------------------------------------------------------------------
// Census 5x5 and downsampling
// ---------------------------------------------------------------------------------------
// Two views per launch: blockIdx.z = 0 uses (img, out), 1 uses (img2, out2).
#ifdef MPV_MISC_KERNELS
__global__ __launch_bounds__(256) void k_census(const uint8_t* __restrict__ img, int W, int H,
                                                int pitch, uint32_t* __restrict__ out,
                                                int opitch, int omargin,
                                                const uint8_t* __restrict__ img2, int pitch2,
                                                uint32_t* __restrict__ out2) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= W || y >= H) return;
  if (blockIdx.z) {
    img = img2;
    pitch = pitch2;
    out = out2;
  }
  const int c = img[(size_t)y * pitch + x];
  uint32_t v = 0;
  int bit = 0;
#pragma unroll
  for (int dy = -2; dy <= 2; ++dy) {
    const int yy = min(max(y + dy, 0), H - 1);
    const uint8_t* row = img + (size_t)yy * pitch;
#pragma unroll
    for (int dx = -2; dx <= 2; ++dx) {
      if (dx == 0 && dy == 0) continue;
      const int xx = min(max(x + dx, 0), W - 1);
      v |= (uint32_t)(row[xx] < c) << bit;
      ++bit;
    }
  }
  out[(size_t)y * opitch + omargin + x] = v;
}
#endif


#ifdef MPV_MISC_KERNELS
__global__ __launch_bounds__(256) void k_downsample(const uint8_t* __restrict__ in, int pitch,
                                                    uint8_t* __restrict__ out, int w, int h,
                                                    const uint8_t* __restrict__ in2, int pitch2,
                                                    uint8_t* __restrict__ out2) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= w || y >= h) return;
  if (blockIdx.z) {
    in = in2;
    pitch = pitch2;
    out = out2;
  }
  const uint8_t* r0 = in + (size_t)(2 * y) * pitch + 2 * x;
  const uint8_t* r1 = r0 + pitch;
  out[(size_t)y * w + x] = (uint8_t)((r0[0] + r0[1] + r1[0] + r1[1] + 2) >> 2);
}
#endif


// ---------------------------------------------------------------------------------------
// Cost volume export: one block per row; both census rows are built in LDS first.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t census_at(const uint8_t* img, int W, int H, int pitch, int x,
                                              int y) {
  const int c = img[(size_t)y * pitch + x];
  uint32_t v = 0;
  int bit = 0;
  for (int dy = -2; dy <= 2; ++dy) {
    const int yy = min(max(y + dy, 0), H - 1);
    for (int dx = -2; dx <= 2; ++dx) {
      if (dx == 0 && dy == 0) continue;
      const int xx = min(max(x + dx, 0), W - 1);
      v |= (uint32_t)(img[(size_t)yy * pitch + xx] < c) << bit;
      ++bit;
    }
  }
  return v;
}

// Pixel (x, y) of the level S halvings below the input: the 2x2 rounded mean applied S
// times (Section 3.4 pyramid), each step over the four pixels of the step below.
template <int S>
__device__ __forceinline__ int pyr_pixel(const uint8_t* img, int pitch, int x, int y) {
  if constexpr (S == 0) {
    return img[(size_t)y * pitch + x];
  } else {
    const int a = pyr_pixel<S - 1>(img, pitch, 2 * x, 2 * y);
    const int b = pyr_pixel<S - 1>(img, pitch, 2 * x + 1, 2 * y);
    const int c = pyr_pixel<S - 1>(img, pitch, 2 * x, 2 * y + 1);
    const int d = pyr_pixel<S - 1>(img, pitch, 2 * x + 1, 2 * y + 1);
    return (a + b + c + d + 2) >> 2;
  }
}

// Census tile `blk` (blocks of every level numbered from level 0, cp.first[]) of view v:
// a 64x4 tile of one level's census. The tile's pixels and a 2-pixel border (coordinates
// clamped to the level, as the census clamps its neighbours) are built in LDS from the
// input, then the block's threads (any multiple of 64) take one census each.
__device__ __forceinline__ void census_pyr_tile(const CenPyr& cp, int blk, int v) {
  __shared__ uint8_t t[8][68];
  const int nt = blockDim.x;
  int l = 0;
  while (l + 1 < cp.L && blk >= cp.first[l + 1]) ++l;
  const int b = blk - cp.first[l];
  const int W = cp.W[l], H = cp.H[l];
  const int x0 = (b % cp.tiles_x[l]) * 64, y0 = (b / cp.tiles_x[l]) * 4;
  const int s = cp.L - 1 - l;
  const uint8_t* img = cp.img[v];
  const int pitch = cp.pitch[v];
  for (int i = threadIdx.x; i < 8 * 68; i += nt) {
    const int ty = i / 68, tx = i % 68;
    const int x = min(max(x0 + tx - 2, 0), W - 1), y = min(max(y0 + ty - 2, 0), H - 1);
    int p;
    if (s == 0) p = pyr_pixel<0>(img, pitch, x, y);
    else if (s == 1) p = pyr_pixel<1>(img, pitch, x, y);
    else if (s == 2) p = pyr_pixel<2>(img, pitch, x, y);
    else p = pyr_pixel<3>(img, pitch, x, y);
    t[ty][tx] = (uint8_t)p;
  }
  __syncthreads();
  for (int o = threadIdx.x; o < 256; o += nt) {
    const int tx = o & 63, ty = o >> 6;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= W || y >= H) continue;
    const int c = t[ty + 2][tx + 2];
    uint32_t val = 0;
    int bit = 0;
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) {
        if (dx == 0 && dy == 0) continue;
        val |= (uint32_t)(t[ty + 2 + dy][tx + 2 + dx] < c) << bit;
        ++bit;
      }
    cp.out[l][v][(size_t)y * cp.opitch[l] + cp.omargin[l] + x] = val;
    if (v == 0 && cp.limg[l]) cp.limg[l][(size_t)y * W + x] = (uint8_t)c;
  }
}

#ifdef MPV_MISC_KERNELS
// Census of every pyramid level of both views in one launch (blockIdx.y = view).
__global__ __launch_bounds__(256) void k_census_pyr(CenPyr cp) {
  census_pyr_tile(cp, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void k_cost(const uint8_t* __restrict__ L, int lpitch,
                                              const uint8_t* __restrict__ R, int rpitch, int W,
                                              int H, const int16_t* __restrict__ lo,
                                              const uint8_t* __restrict__ len, int cap, int D,
                                              uint8_t* __restrict__ cost) {
  extern __shared__ uint32_t s_cen[];  // [2][W]
  const int y = blockIdx.x;
  for (int x = threadIdx.x; x < W; x += blockDim.x) {
    s_cen[x] = census_at(L, W, H, lpitch, x, y);
    s_cen[W + x] = census_at(R, W, H, rpitch, x, y);
  }
  __syncthreads();
  const size_t n = (size_t)W * cap;
  uint8_t* row = cost + (size_t)y * n;
  for (size_t i = threadIdx.x; i < n; i += blockDim.x) {
    const int x = (int)(i / cap), j = (int)(i % cap);
    const size_t p = (size_t)y * W + x;
    int b0, bn;
    band_at(lo, len, p, D, cap, b0, bn);
    uint8_t c = 0xFF;
    if (j < bn) {
      const int d = b0 + j;
      c = (x - d >= 0) ? (uint8_t)__popc(s_cen[x] ^ s_cen[W + x - d]) : (uint8_t)24;
    }
    row[i] = c;
  }
}
#endif


// ---------------------------------------------------------------------------------------
// Scan kernels
// ---------------------------------------------------------------------------------------






// Descriptor index of global unit u (binary search; all lanes agree).
__device__ __forceinline__ int batch_find(const int* first, int nseg, int u) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= u)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Wave index of this wave in a launch whose blocks hold blockDim.x / 64 waves.
__device__ __forceinline__ int wave_unit() {
  return __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
}

// True when `c` holds in every lane of the wave (all lanes active).
__device__ __forceinline__ bool wave_all(bool c) { return __builtin_amdgcn_ballot_w64(!c) == 0; }

__device__ __forceinline__ int num_lines(int r, int W, int H) {
  return c_dy[r] == 0 ? H : (c_dx[r] == 0 ? W : W + H - 1);
}

// First pixel and length of line i of direction r. Lines start where p - r leaves the image.
__device__ __forceinline__ void line_info(int r, int i, int W, int H, int& x0, int& y0, int& n) {
  const int dx = c_dx[r], dy = c_dy[r];
  if (dy == 0) {
    y0 = i;
    x0 = dx > 0 ? 0 : W - 1;
    n = W;
  } else if (dx == 0) {
    x0 = i;
    y0 = dy > 0 ? 0 : H - 1;
    n = H;
  } else {
    if (i < W) {
      x0 = i;
      y0 = dy > 0 ? 0 : H - 1;
    } else {
      const int k = i - W + 1;
      x0 = dx > 0 ? 0 : W - 1;
      y0 = dy > 0 ? k : H - 1 - k;
    }
    const int nx = dx > 0 ? W - x0 : x0 + 1;
    const int ny = dy > 0 ? H - y0 : y0 + 1;
    n = min(nx, ny);
  }
}

// One Viterbi line: first pixel, step, length (group-uniform).
struct Line {
  int x0, y0, dx, dy, n;
};

// Pixel of step t (clamped to the line so that finished or empty lines stay in bounds).
__device__ __forceinline__ size_t line_pixel(const Line& ln, int t, int W, int& x, int& y) {
  const int tt = t < ln.n ? t : (ln.n > 0 ? ln.n - 1 : 0);
  x = ln.x0 + tt * ln.dx;
  y = ln.y0 + tt * ln.dy;
  return (size_t)y * W + x;
}

// Wave unit b of a descriptor -> (direction, this group's line); nmax = longest line of the wave.
template <int LPL>
__device__ __forceinline__ void block_line(const ScanArgs& a, int b, int& r, int& ri, Line& ln,
                                           int& nmax) {
  ri = 0;
  while (ri + 1 < a.ndir && b >= a.gprefix[ri + 1]) ++ri;
  r = a.dir[ri];
  ln.dx = c_dx[r];
  ln.dy = c_dy[r];
  const int g = LPL == 64 ? 0 : lane_id() / LPL;  // 64-lane groups: wave-uniform line data
  const int line = (b - a.gprefix[ri]) * (64 / LPL) + g;
  if (line < num_lines(r, a.W, a.H)) {
    line_info(r, line, a.W, a.H, ln.x0, ln.y0, ln.n);
  } else {
    ln.x0 = 0;
    ln.y0 = 0;
    ln.n = 0;
  }
  nmax = __builtin_amdgcn_readfirstlane(ln.n);
#pragma unroll
  for (int k = 1; k < 64 / LPL; ++k) nmax = max(nmax, __builtin_amdgcn_readlane(ln.n, k * LPL));
}

// Compile-time loop: f(std::integral_constant<int, 0>) ... f(<N-1>).
template <typename F, int... Is>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Lane K of each LPL-lane group, broadcast to the group (K < 16).
template <int LPL, int K>
__device__ __forceinline__ int group_bcast(int v) {
  if constexpr (LPL == 64)
    return __builtin_amdgcn_readlane(v, K);
  else if constexpr (LPL == 32)
    return __builtin_amdgcn_ds_swizzle(v, K << 5);
  else
    return __builtin_amdgcn_ds_swizzle(v, 0x10 | (K << 5));
}

// Per-step line data, staged a chunk at a time: lane k of a group holds step t0+k as one
// packed word (left census in bits 0..23, band start in bits 24..31; D <= 256) plus, for
// variable-length bands, the band length. Words are broadcast to the group PREFETCH steps
// ahead of use, together with the per-lane right-census loads of that step.
constexpr int CHUNK = 16;
constexpr int PREFETCH = 4;

// 32-bit offsets of step t's pixel along a line (clamped to the line).
// 32-bit load at a byte offset from a uniform base (lets the compiler use scalar-base
// addressing with a 32-bit vector offset)
__device__ __forceinline__ uint32_t ld_u32(const uint32_t* base, uint32_t idx) {
  return *(const uint32_t*)((const char*)base + (idx << 2));
}

struct LineAddr {
  int n;
  int x0, dx;  // x
  int p0, dp;  // y*W + x
  int c0, dc;  // census offset y*cpitch + cmargin + x
  int i0, di;  // left image offset y*ipitch + x (gradient-weighted transitions)
  __device__ __forceinline__ int tt(int t) const { return min(t, max(n - 1, 0)); }
  // offsets are non-negative and below 2^32: unsigned 32-bit, added to uniform bases
  __device__ __forceinline__ uint32_t pix(int t) const { return (uint32_t)(p0 + tt(t) * dp); }
  __device__ __forceinline__ uint32_t cen(int t) const { return (uint32_t)(c0 + tt(t) * dc); }
};

__device__ __forceinline__ LineAddr line_addr(const ScanArgs& a, const Line& ln) {
  LineAddr la;
  la.n = ln.n;
  la.x0 = ln.x0;
  la.dx = ln.dx;
  la.p0 = ln.y0 * a.W + ln.x0;
  la.dp = ln.dy * a.W + ln.dx;
  la.c0 = ln.y0 * a.cpitch + a.cmargin + ln.x0;
  la.dc = ln.dy * a.cpitch + ln.dx;
  la.i0 = ln.y0 * a.ipitch + ln.x0;
  la.di = ln.dy * a.ipitch + ln.dx;
  return la;
}

template <bool BANDED, int SRC>
__device__ __forceinline__ uint2 load_chunk(const ScanArgs& a, const LineAddr& la, int t0, int k) {
  int b0 = 0, bn = a.D;
  if constexpr (BANDED) band_at(a.lo, a.len, (size_t)la.pix(t0 + k), a.D, a.cap, b0, bn);
  const uint32_t cl = src_census(SRC) ? ld_u32(a.cl, la.cen(t0 + k)) : 0u;
  uint32_t y = (uint32_t)bn;
  if constexpr (src_grad(SRC)) {
    // weight of the edge from step t-1 to step t (eq. EU), in bits 16..23 beside the band
    // length; double precision, so the rounding matches any correctly rounded exp
    const int t = la.tt(t0 + k);
    const int g = abs((int)a.img[la.i0 + t * la.di] - (int)a.img[la.i0 + max(t - 1, 0) * la.di]);
    const int w = (int)floor((double)a.lambda * exp(-(double)g / (double)a.sigma) + 0.5);
    y |= (uint32_t)w << 16;
  }
  return make_uint2(cl | ((uint32_t)b0 << 24), y);
}

// Packed-pair shift of the disparity axis by s (s = 1 or even s) inside the group.
// up: value from d - s; down: value from d + s. Lane l holds pairs of d = 2(lK+k), +1.
template <int LPL, int K>
__device__ __forceinline__ void shift_pairs_up(const uint32_t (&v)[K], uint32_t (&o)[K], int s) {
  if (s == 1) {
    const uint32_t prev = from_prev_lane<LPL>(v[K - 1], INF2);
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] = funnel16(v[k], k ? v[k - 1] : prev);
  } else {
    const int q = s >> 1;
    const int loff = q / K, rem = q % K;
    uint32_t a[K], b[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      a[k] = shift_up<LPL>(v[k], loff, INF2);
      b[k] = shift_up<LPL>(v[k], loff + 1, INF2);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int kk = k - rem;
      o[k] = kk >= 0 ? a[kk >= 0 ? kk : 0] : b[kk + K >= 0 ? kk + K : 0];
    }
  }
}

template <int LPL, int K>
__device__ __forceinline__ void shift_pairs_down(const uint32_t (&v)[K], uint32_t (&o)[K], int s) {
  if (s == 1) {
    const uint32_t next = from_next_lane<LPL>(v[0], INF2);
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] = funnel16(k + 1 < K ? v[k + 1] : next, v[k]);
  } else {
    const int q = s >> 1;
    const int loff = q / K, rem = q % K;
    uint32_t a[K], b[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      a[k] = shift_down<LPL>(v[k], loff, INF2);
      b[k] = shift_down<LPL>(v[k], loff + 1, INF2);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int kk = k + rem;
      o[k] = kk < K ? a[kk < K ? kk : 0] : b[kk - K < K ? kk - K : 0];
    }
  }
}

// Compile-time version of the packed-pair shifts (S = 1 or even S).
template <int LPL, int K, int S>
__device__ __forceinline__ void shift_pairs_up_c(const uint32_t (&v)[K], uint32_t (&o)[K]) {
  if constexpr (S == 1) {
    const uint32_t prev = from_prev_lane<LPL>(v[K - 1], INF2);
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] = funnel16(v[k], k ? v[k - 1] : prev);
  } else {
    constexpr int q = S / 2, loff = q / K, rem = q % K;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k - rem >= 0)
        o[k] = shift_up_c<LPL, loff>(v[k - rem >= 0 ? k - rem : 0], INF2);
      else
        o[k] = shift_up_c<LPL, loff + 1>(v[k - rem + K], INF2);
    }
  }
}

template <int LPL, int K, int S>
__device__ __forceinline__ void shift_pairs_down_c(const uint32_t (&v)[K], uint32_t (&o)[K]) {
  if constexpr (S == 1) {
    const uint32_t next = from_next_lane<LPL>(v[0], INF2);
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] = funnel16(k + 1 < K ? v[k + 1] : next, v[k]);
  } else {
    constexpr int q = S / 2, loff = q / K, rem = q % K;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k + rem < K)
        o[k] = shift_down_c<LPL, loff>(v[k + rem < K ? k + rem : 0], INF2);
      else
        o[k] = shift_down_c<LPL, loff + 1>(v[k + rem - K], INF2);
    }
  }
}

// Envelope min_{|k|<tau} P(d+k) + lambda|k| of packed pairs by doubling sweeps
// (TAU > 0: compile-time tau; TAU == 0: runtime tau).
// lam_up weighs the sweep from lower disparities (an increase along the path), lambda the
// sweep from higher ones.
template <int LPL, int K, int TAU>
__device__ __forceinline__ void pair_envelope(const uint32_t (&P)[K], uint32_t (&E)[K], int tau,
                                              int lambda, int lam_up) {
  uint32_t A[K], B[K], T[K];
#pragma unroll
  for (int q = 0; q < K; ++q) A[q] = B[q] = P[q];
  if constexpr (TAU > 0) {
    static_for<ceil_log2(TAU)>([&](auto ic) {
      constexpr int S = 1 << decltype(ic)::value;
      const uint32_t pen = splat16((uint32_t)(S * lambda));
      const uint32_t pup = splat16((uint32_t)(S * lam_up));
      shift_pairs_up_c<LPL, K, S>(A, T);
#pragma unroll
      for (int q = 0; q < K; ++q) A[q] = pk_min(A[q], pk_add(T[q], pup));
      shift_pairs_down_c<LPL, K, S>(B, T);
#pragma unroll
      for (int q = 0; q < K; ++q) B[q] = pk_min(B[q], pk_add(T[q], pen));
    });
  } else {
    for (int s = 1; s < tau; s <<= 1) {
      const uint32_t pen = splat16((uint32_t)(s * lambda));
      const uint32_t pup = splat16((uint32_t)(s * lam_up));
      shift_pairs_up<LPL, K>(A, T, s);
#pragma unroll
      for (int q = 0; q < K; ++q) A[q] = pk_min(A[q], pk_add(T[q], pup));
      shift_pairs_down<LPL, K>(B, T, s);
#pragma unroll
      for (int q = 0; q < K; ++q) B[q] = pk_min(B[q], pk_add(T[q], pen));
    }
  }
#pragma unroll
  for (int q = 0; q < K; ++q) E[q] = pk_min(A[q], B[q]);
}

// Band envelope in the previous pixel's frame extended by tau-1 lanes on each side.
template <int LPL, int TAU>
__device__ __forceinline__ uint32_t band_envelope(uint32_t P, int tau, int lambda, int lam_up) {
  if constexpr (TAU > 0) {
    uint32_t A = shift_up_c<LPL, TAU - 1>(P, INF32);
    uint32_t B = A;
    static_for<ceil_log2(TAU)>([&](auto ic) {
      constexpr int S = 1 << decltype(ic)::value;
      A = min(A, shift_up_c<LPL, S>(A, INF32) + (uint32_t)(S * lam_up));
      B = min(B, shift_down_c<LPL, S>(B, INF32) + (uint32_t)(S * lambda));
    });
    return min(A, B);
  } else {
    uint32_t A = shift_up<LPL>(P, tau - 1, INF32);
    uint32_t B = A;
    for (int s = 1; s < tau; s <<= 1) {
      A = min(A, shift_up<LPL>(A, s, INF32) + (uint32_t)(s * lam_up));
      B = min(B, shift_down<LPL>(B, s, INF32) + (uint32_t)(s * lambda));
    }
    return min(A, B);
  }
}

// Complement-encoded packed-pair shifts (zero fill = absent) and envelope, compile-time TAU.
template <int LPL, int K, int S>
__device__ __forceinline__ void zshift_pairs_up(const uint32_t (&v)[K], uint32_t (&o)[K]) {
  if constexpr (S == 1) {
    const uint32_t prev = (uint32_t)zshift_up<LPL, 1>((int)v[K - 1]);
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] = funnel16(v[k], k ? v[k - 1] : prev);
  } else {
    constexpr int q = S / 2, loff = q / K, rem = q % K;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k - rem >= 0)
        o[k] = (uint32_t)zshift_up<LPL, loff>((int)v[k - rem >= 0 ? k - rem : 0]);
      else
        o[k] = (uint32_t)zshift_up<LPL, loff + 1>((int)v[k - rem + K]);
    }
  }
}

template <int LPL, int K, int S>
__device__ __forceinline__ void zshift_pairs_down(const uint32_t (&v)[K], uint32_t (&o)[K]) {
  if constexpr (S == 1) {
    const uint32_t next = (uint32_t)zshift_down<LPL, 1>((int)v[0]);
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] = funnel16(k + 1 < K ? v[k + 1] : next, v[k]);
  } else {
    constexpr int q = S / 2, loff = q / K, rem = q % K;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k + rem < K)
        o[k] = (uint32_t)zshift_down<LPL, loff>((int)v[k + rem < K ? k + rem : 0]);
      else
        o[k] = (uint32_t)zshift_down<LPL, loff + 1>((int)v[k + rem - K]);
    }
  }
}

// max over |k| < TAU of u(d+k) - lambda|k| for packed complement pairs.
template <int LPL, int K, int TAU>
__device__ __forceinline__ void pair_envelope_c(const uint32_t (&Pu)[K], uint32_t (&E)[K],
                                                int lambda, int lam_up) {
  uint32_t A[K], B[K], X[K], T[K];
#pragma unroll
  for (int q = 0; q < K; ++q) A[q] = B[q] = Pu[q];
  static_for<ceil_log2(TAU)>([&](auto ic) {
    constexpr int S = 1 << decltype(ic)::value;
    const uint32_t pen = splat16((uint32_t)(S * lambda));
    const uint32_t pup = splat16((uint32_t)(S * lam_up));
#pragma unroll
    for (int q = 0; q < K; ++q) X[q] = pk_sub_i(A[q], pup);
    zshift_pairs_up<LPL, K, S>(X, T);
#pragma unroll
    for (int q = 0; q < K; ++q) A[q] = pk_max_i(A[q], T[q]);
#pragma unroll
    for (int q = 0; q < K; ++q) X[q] = pk_sub_i(B[q], pen);
    zshift_pairs_down<LPL, K, S>(X, T);
#pragma unroll
    for (int q = 0; q < K; ++q) B[q] = pk_max_i(B[q], T[q]);
  });
#pragma unroll
  for (int q = 0; q < K; ++q) E[q] = pk_max_i(A[q], B[q]);
}

// Complement-encoded band envelope for compile-time TAU (u = INF32 - value, absent = 0):
// max over |k| < TAU of u(i+k) - lambda|k| in the previous pixel's frame extended by
// TAU-1 lanes on each side. Absent nodes stay <= 0 < every present node.
template <int LPL, int TAU>
__device__ __forceinline__ int band_envelope_c(int Pu, int lambda, int lam_up) {
  int A = zshift_up<LPL, TAU - 1>(Pu);
  int B = A;
  static_for<ceil_log2(TAU)>([&](auto ic) {
    constexpr int S = 1 << decltype(ic)::value;
    A = max(A, zshift_up<LPL, S>(A - S * lam_up));
    B = max(B, zshift_down<LPL, S>(B - S * lambda));
  });
  return max(A, B);
}

// ---- suffix extrema along the disparity axis (occlusion weight of the layered merge:
// every predecessor at least tau above d costs lambda*tau, at least tau below 2*lambda*tau,
// so the truncation candidate needs the best predecessor at or above d).
// Complement-encoded (absent 0): lane i of the group gets the maximum over lanes >= i.
template <int LPL>
__device__ __forceinline__ int suffix_max_lanes(int v) {
  static_for<ceil_log2(LPL)>([&](auto ic) {
    constexpr int S = 1 << decltype(ic)::value;
    v = max(v, zshift_down<LPL, S>(v));
  });
  return v;
}
// Plain energies: the minimum over lanes >= i, `fill` beyond the group.
template <int LPL>
__device__ __forceinline__ uint32_t suffix_min_lanes(uint32_t v, uint32_t fill) {
  static_for<ceil_log2(LPL)>([&](auto ic) {
    constexpr int S = 1 << decltype(ic)::value;
    v = min(v, shift_down_c<LPL, S>(v, fill));
  });
  return v;
}
// Packed pairs (lane l holds d = 2(lK+q), +1): suffix maximum of complement energies.
template <int LPL, int K>
__device__ __forceinline__ void pair_suffix_max_c(const uint32_t (&v)[K], uint32_t (&o)[K]) {
  int run = 0;
#pragma unroll
  for (int q = K - 1; q >= 0; --q) {
    const int hi = max(hi16s(v[q]), run);
    const int lo = max(lo16s(v[q]), hi);
    o[q] = ((uint32_t)lo & 0xFFFFu) | ((uint32_t)hi << 16);
    run = lo;
  }
  const int above = zshift_down<LPL, 1>(suffix_max_lanes<LPL>(run));  // lanes above this one
  const uint32_t ab = splat16((uint32_t)above & 0xFFFFu);
#pragma unroll
  for (int q = 0; q < K; ++q) o[q] = pk_max_i(o[q], ab);
}
// Packed pairs: suffix minimum of plain 16-bit energies (absent >= INF16).
template <int LPL, int K>
__device__ __forceinline__ void pair_suffix_min(const uint32_t (&v)[K], uint32_t (&o)[K]) {
  uint32_t run = INF16;
#pragma unroll
  for (int q = K - 1; q >= 0; --q) {
    const uint32_t hi = min(hi16(v[q]), run);
    const uint32_t lo = min(lo16(v[q]), hi);
    o[q] = lo | (hi << 16);
    run = lo;
  }
  const uint32_t above = shift_down_c<LPL, 1>(suffix_min_lanes<LPL>(run, INF16), INF16);
  const uint32_t ab = splat16(above);
#pragma unroll
  for (int q = 0; q < K; ++q) o[q] = pk_min(o[q], ab);
}

template <int OUT>
__device__ __forceinline__ void export_canonical(void* agg, size_t idx, uint32_t v, int first) {
  if constexpr (OUT == OUT_U16) {
    uint16_t* s = (uint16_t*)agg + idx;
    *s = first ? (uint16_t)v : (uint16_t)(*s + v);
  } else {
    int32_t* s = (int32_t*)agg + idx;
    *s = first ? (int32_t)v : (int32_t)(*s + v);
  }
}

// Full-range scan. Template: LPL lanes per line, K packed pairs per lane (D <= 2*K*LPL),
// SRC census (fused cost) or a cost volume, OUT normalised uint8 partial or canonical
// (unnormalised) export, TAU compile-time tau (0: runtime). BANDED: a lane's disparity
// outside the pixel's band is an absent node; partials are then indexed by absolute
// disparity.
// `a`: the descriptor's values; `tab`: the same descriptor where its direction tables are
// read (batched launches pass a private copy as `a` and the table entry as `tab`).
template <int LPL, int K, int SRC, int OUT, int TAU, bool BANDED>
__device__ __forceinline__ void scan_full_wave(const ScanArgs& a, const ScanArgs& tab, int unit) {
  const int lane = lane_id();
  const int l = LPL == 64 ? lane : lane % LPL;
  const int kk = l % CHUNK;
  int r, ri, nmax;
  Line ln;
  block_line<LPL>(tab, unit, r, ri, ln, nmax);
  const LineAddr la = line_addr(a, ln);
  const uint32_t lt = (uint32_t)(a.lambda * a.tau);
  // occlusion weight of the layered merge: this direction pays 2*lambda per disparity step up
  const bool occ = src_occ(SRC) && r == a.up_dir;
  constexpr bool GRAD = src_grad(SRC);
  uint32_t P[K];
#pragma unroll
  for (int k = 0; k < K; ++k) P[k] = 0;
  uint32_t acc = 0;  // canonical offset: sum of the minima subtracted so far
  uint8_t* part = a.part + (long long)(a.dir_base + ri) * a.part_stride;
  uint8_t* const sinkp = a.part + (long long)a.npd * a.part_stride;  // 256 B behind the volumes
  const rsrc_t rpart = make_rsrc(part);

  // The lane's NC candidates d0l .. d0l+NC-1 sit at census offsets c-d0l-NC+1 .. c-d0l:
  // element i of a fetch is the right census of d = d0l + NC-1-i. For 64-lane groups c is
  // wave-uniform, so the base is scalar and the lane offset a constant.
  constexpr int NC = 2 * K, SPAN = 2 * LPL * K;
  const int d0l = 2 * l * K;
  const uint32_t loff = (uint32_t)(SPAN - d0l - NC) << 2;
  uint32_t ring[PREFETCH][NC];  // right census of the lane's NC candidates
  uint32_t bw[PREFETCH];        // broadcast step words
  int bl[PREFETCH];             // broadcast band lengths
  const rsrc_t rcr = make_rsrc(a.cr);
  // SRC_MERGE: the lane's 2K slots of both source volumes, loaded PREFETCH steps ahead.
  // off = the step's pixel index times capP; uni: off is wave-uniform (scalar offset).
  const rsrc_t rmA = make_rsrc(src_merge(SRC) ? a.msrc : a.part);
  const rsrc_t rmB = make_rsrc(src_merge(SRC) ? a.msrc + a.part_stride : a.part);
  uint32_t mring[PREFETCH][2];
  auto fetch_m = [&](uint32_t off, bool uni, uint32_t (&dst)[2]) {
    if constexpr (src_merge(SRC)) {
      const uint32_t vo = uni ? (uint32_t)(2 * l * K) : off + 2 * l * K, so = uni ? off : 0u;
      if constexpr (K == 1) {
        dst[0] = buf_ld16(rmA, vo, so);
        dst[1] = buf_ld16(rmB, vo, so);
      } else {
        dst[0] = buf_ld32(rmA, vo, so);
        dst[1] = buf_ld32(rmB, vo, so);
      }
    }
  };
  auto fetch_c = [&](uint32_t c, uint32_t (&dst)[NC]) {
    if constexpr (src_census(SRC)) {
      // c >= census margin > SPAN, so every offset below is non-negative
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        if constexpr (LPL == 64)
          dst[i] = buf_ld32(rcr, loff + 4 * i, (c - (uint32_t)(SPAN - 1)) << 2);
        else
          dst[i] = buf_ld32(rcr, ((c - (uint32_t)(d0l + NC - 1)) << 2) + 4 * i, 0u);
      }
    }
  };
  uint2 cur = load_chunk<BANDED, SRC>(a, la, 0, kk);
  static_for<PREFETCH>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    bw[q] = (uint32_t)group_bcast<LPL, q>((int)cur.x);
    if constexpr (BANDED || GRAD) bl[q] = group_bcast<LPL, q>((int)cur.y);
    fetch_c(la.cen(q), ring[q]);
    fetch_m(la.pix(q) * (uint32_t)a.capP, false, mring[q]);
  });
  // loop-invariant masks: halves for d >= D are absent nodes (unbanded path)
  uint32_t dmask[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int d0 = d0l + 2 * q;
    dmask[q] = (d0 < a.D ? 0u : INF16) | ((d0 + 1 < a.D ? 0u : INF16) << 16);
  }
  const uint32_t pstep = (uint32_t)(la.dp * a.capP);

  // One step. FAST: the whole chunk and its prefetches lie inside every line of the wave and
  // every candidate has x - d >= 0, so offsets run incrementally with no clamps or border tests.
  auto step = [&](auto kc, auto fc, const uint2& nxt, int t0, uint32_t pst, uint32_t cpf) {
    constexpr int k = decltype(kc)::value;
    constexpr bool FAST = decltype(fc)::value;
    constexpr int slot = k % PREFETCH;
    const int t = t0 + k;
    const uint32_t w = bw[slot];
    const int b0 = BANDED ? (int)(w >> 24) : 0;
    const int bn = BANDED ? (GRAD ? bl[slot] & 0xFFFF : bl[slot]) : a.D;
    // transition weight of this step: lambda, or the edge's gradient weight (eq. EU)
    const int lam_s = GRAD ? (int)((uint32_t)bl[slot] >> 16) : a.lambda;
    const uint32_t lt_s = GRAD ? (uint32_t)(lam_s * a.tau) : lt;
    const int lam_up = occ ? 2 * lam_s : lam_s;
    uint32_t cr[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) cr[q] = ring[slot][q];
    const uint32_t mA = mring[slot][0], mB = mring[slot][1];
    {  // step t + PREFETCH: broadcast its word and issue its census (or source) loads
      constexpr int kn = (k + PREFETCH) % CHUNK;
      const uint2 src = k + PREFETCH < CHUNK ? cur : nxt;
      bw[slot] = (uint32_t)group_bcast<LPL, kn>((int)src.x);
      if constexpr (BANDED || GRAD) bl[slot] = group_bcast<LPL, kn>((int)src.y);
      fetch_c(FAST ? cpf : la.cen(t + PREFETCH), ring[slot]);
      fetch_m(FAST ? pst + (uint32_t)PREFETCH * pstep : la.pix(t + PREFETCH) * (uint32_t)a.capP,
              FAST && LPL == 64, mring[slot]);
    }
    // ---- matching cost of this pixel, two disparities per pair
    uint32_t C[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const int d0 = d0l + 2 * q;
      uint32_t c0, c1;
      if constexpr (src_census(SRC)) {
        const uint32_t cl = w & 0xFFFFFFu;
        c0 = (uint32_t)__popc(cl ^ cr[NC - 1 - 2 * q]);
        c1 = (uint32_t)__popc(cl ^ cr[NC - 2 - 2 * q]);
        if constexpr (!FAST) {
          const int x = la.x0 + la.tt(t) * la.dx;
          c0 = (x - d0 >= 0) ? c0 : 24u;
          c1 = (x - d0 - 1 >= 0) ? c1 : 24u;
        }
      } else if constexpr (src_merge(SRC)) {
        // bytes 2q, 2q+1 of both sources as a 16-bit pair, merged per node
        const uint32_t sel = 0x0c000c00u | ((uint32_t)(2 * q + 1) << 16) | (uint32_t)(2 * q);
        const uint32_t ua = __builtin_amdgcn_perm(0u, mA, sel), ub = __builtin_amdgcn_perm(0u, mB, sel);
        const uint32_t cm = a.mop == MERGE_MEAN ? ((ua + ub) >> 1) & 0x7FFF7FFFu : pk_min(ua, ub);
        c0 = cm & 0xFFFFu;
        c1 = cm >> 16;
      } else {
        const uint8_t* cp = a.cost + (size_t)la.pix(t) * a.cap;
        const int j0 = min(max(d0 - b0, 0), a.cap - 1), j1 = min(max(d0 + 1 - b0, 0), a.cap - 1);
        c0 = cp[j0];
        c1 = cp[j1];
      }
      if constexpr (BANDED) {
        const bool in0 = d0 < a.D && d0 >= b0 && d0 < b0 + bn;
        const bool in1 = d0 + 1 < a.D && d0 + 1 >= b0 && d0 + 1 < b0 + bn;
        C[q] = (in0 ? c0 : INF16) | ((in1 ? c1 : INF16) << 16);
      } else {
        C[q] = pk_max(c0 | (c1 << 16), dmask[q]);
      }
    }
    // ---- transition: min over predecessors of P(d') + lambda*min(|d-d'|, tau),
    //      then normalise by the minimum over the line's disparities
    uint32_t L[K];
    uint32_t m;
    if constexpr (TAU > 0) {
      // complement encoding (u = INF16 - value per half, absent <= 0): max instead of min
      uint32_t E[K];
      pair_envelope_c<LPL, K, TAU>(P, E, lam_s, lam_up);
      const uint32_t cap = t == 0 ? INF2 : splat16(INF16 - lt_s);
      uint32_t capq[K];
#pragma unroll
      for (int q = 0; q < K; ++q) capq[q] = cap;
      if constexpr (src_occ(SRC)) {
        if (occ && t != 0) {  // the previous minimum + 2*lambda*tau, the best at or above d + lambda*tau
          uint32_t SU[K];
          pair_suffix_max_c<LPL, K>(P, SU);
#pragma unroll
          for (int q = 0; q < K; ++q)
            capq[q] = pk_max_i(splat16(INF16 - 2 * lt_s), pk_sub_i(SU[q], splat16(lt_s)));
        }
      }
      int mu = -32768;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        L[q] = pk_sub_i(pk_max_i(E[q], capq[q]), C[q]);
        mu = max(mu, max(lo16s(L[q]), hi16s(L[q])));
      }
      if constexpr (LPL == 64)
        mu = wave_max_s(mu);  // scalar: the splats below are scalar too
      else
        mu = group_max<LPL>(mu);
      m = INF16 - (uint32_t)mu;
      const uint32_t off = splat16(m);
#pragma unroll
      for (int q = 0; q < K; ++q) {
        P[q] = pk_add_i(L[q], off);  // next state, complement encoded
        if constexpr (OUT == OUT_PART)
          L[q] = pk_sub_i(splat16((uint32_t)mu), L[q]);  // energy minus the line minimum
        else
          L[q] = pk_sub_i(INF2, L[q]);  // energies relative to the previous minimum
      }
    } else {
      uint32_t E[K];
      pair_envelope<LPL, K, TAU>(P, E, a.tau, lam_s, lam_up);
      const uint32_t mcap = t == 0 ? 0u : splat16(lt_s);  // the first pixel has no predecessor
      uint32_t mc[K];
#pragma unroll
      for (int q = 0; q < K; ++q) mc[q] = mcap;
      if constexpr (src_occ(SRC)) {
        if (occ && t != 0) {  // the previous minimum (0) + 2*lambda*tau, the best at or above d + lambda*tau
          uint32_t SM[K];
          pair_suffix_min<LPL, K>(P, SM);
#pragma unroll
          for (int q = 0; q < K; ++q) mc[q] = pk_min(splat16(2 * lt_s), pk_add(SM[q], splat16(lt_s)));
        }
      }
#pragma unroll
      for (int q = 0; q < K; ++q) L[q] = pk_add(C[q], pk_min(E[q], mc[q]));
      m = min(lo16(L[0]), hi16(L[0]));
#pragma unroll
      for (int q = 1; q < K; ++q) m = min(m, min(lo16(L[q]), hi16(L[q])));
      m = group_min<LPL>(m);
#pragma unroll
      for (int q = 0; q < K; ++q) P[q] = pk_sub(L[q], splat16(m));
    }
    // ---- outputs
    if constexpr (OUT == OUT_PART) {
      // past the line's end the store goes to a sink behind the last direction's volume
      uint32_t v = 0;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const uint32_t nq = TAU > 0 ? L[q] : P[q];  // L - min, >= 0
        const uint32_t c = pk_min(nq, 0x00FF00FFu);
        v |= __builtin_amdgcn_perm(0u, c, 0x0c0c0200u) << (16 * q);
      }
      if constexpr (FAST) {
        // pst is wave-uniform for 64-lane groups: scalar offset, constant lane offset
        const uint32_t vo = LPL == 64 ? 2 * l * K : pst + 2 * l * K, so = LPL == 64 ? pst : 0u;
        if constexpr (K == 1)
          __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, rpart, (int)vo, (int)so, kPartStorePolicy);
        else
          __builtin_amdgcn_raw_buffer_store_b32(v, rpart, (int)vo, (int)so, kPartStorePolicy);
      } else {
        // past the line's end the store goes to a sink behind the last direction's volume
        uint8_t* dst = t < la.n ? part + la.pix(t) * (uint32_t)a.capP + 2 * l * K : sinkp + 4 * lane;
        if constexpr (K == 1)
          *(uint16_t*)dst = (uint16_t)v;
        else
          *(uint32_t*)dst = v;
      }
    } else {
      if (t < la.n) {
        const uint32_t p = la.pix(t);
#pragma unroll
        for (int q = 0; q < K; ++q) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int d = d0l + 2 * q + h;
            const int j = d - b0;
            if (d < a.D && j >= 0 && j < bn)
              export_canonical<OUT>(a.agg, (size_t)p * a.cap + j, (h ? hi16(L[q]) : lo16(L[q])) + acc,
                                    a.first);
          }
        }
      }
    }
    acc += m;
  };

  for (int t0 = 0; t0 < nmax; t0 += CHUNK) {
    const uint2 nxt = load_chunk<BANDED, SRC>(a, la, t0 + CHUNK, kk);
    const int xa = la.x0 + t0 * la.dx, xb = xa + (CHUNK - 1) * la.dx;
    const bool fast = wave_all(t0 + CHUNK + PREFETCH <= la.n &&
                               (!src_census(SRC) || min(xa, xb) >= a.D - 1));
    if (fast) {
      uint32_t pst = (uint32_t)(la.p0 + t0 * la.dp) * (uint32_t)a.capP;
      uint32_t cpf = (uint32_t)(la.c0 + (t0 + PREFETCH) * la.dc);
      static_for<CHUNK>([&](auto kc) {
        step(kc, std::true_type{}, nxt, t0, pst, cpf);
        pst += pstep;
        cpf += (uint32_t)la.dc;
      });
    } else {
      static_for<CHUNK>([&](auto kc) { step(kc, std::false_type{}, nxt, t0, 0u, 0u); });
    }
    cur = nxt;
  }
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Slots 0..9 of a pixel's staged bytes in the six-bit layout (PART6_PITCH): each byte's low
// six bits (the slots past the band hold 255, read as 63 and never summed).
__device__ __forceinline__ u32x2 pack6_bytes(const uint4 v) {
  const uint32_t b[3] = {v.x, v.y, v.z};
  u32x2 w = {0u, 0u};
#pragma unroll
  for (int i = 0; i < PART6_SLOTS; ++i) w[i / 5] |= ((b[i / 4] >> (8 * (i % 4))) & 63u) << (6 * (i % 5));
  return w;
}

// Banded scan: each pixel searches cap < LPL - 2(tau-1) consecutive disparities starting
// at lo(p); lane j holds d = lo(p) + j. Neighbouring pixels may place their bands
// anywhere, so the envelope is built in the previous pixel's frame extended by tau-1
// slots on each side, then lane j of the new pixel picks position j + lo(p) - lo(p-r).
// VAR: per-pixel band lengths (otherwise every pixel has len = cap).
template <int LPL, int SRC, int OUT, int TAU, bool VAR, bool STAGED = false>
__device__ __forceinline__ void scan_band_wave(const ScanArgs& a, const ScanArgs& tab, int unit) {
  const int lane = lane_id();
  const int j = LPL == 64 ? lane : lane % LPL;
  const int kk = j % CHUNK;
  const int gbase = lane - j;
  int r, ri, nmax;
  Line ln;
  block_line<LPL>(tab, unit, r, ri, ln, nmax);
  const LineAddr la = line_addr(a, ln);
  const int e = a.tau - 1;
  const uint32_t lt = (uint32_t)(a.lambda * a.tau);
  // occlusion weight of the layered merge: this direction pays 2*lambda per disparity step up
  const bool occ = src_occ(SRC) && r == a.up_dir;
  constexpr bool GRAD = src_grad(SRC);
  constexpr bool BL = VAR || GRAD;  // the second step word (band length, weight) is broadcast
  uint32_t P = INF32;  // normalised energies of the previous pixel (runtime-tau path)
  // compile-time-tau path: unnormalised energies in complement encoding, Pu = INF32 - L
  // (absent 0). L never needs normalising here: the fused path has data terms plus
  // lambda*tau of at most 255 and lines of at most MPV_MAX_HEIGHT (or MPV_MAX_WIDTH) pixels, so L < 2^24, far from
  // INF32. The line maximum then feeds only the next step's truncation candidate and the
  // stored bytes, off the step's dependent chain.
  int Pu = 0;
  int capu = 0;  // max over the previous pixel's band of Pu, minus lambda*tau
  int mprev = 0;  // max over the previous pixel's band of Pu (gradient weights: per step)
  int lo_prev = 0;
  uint32_t acc = 0;
  uint8_t* part = a.part + (long long)(a.dir_base + ri) * a.part_stride;
  uint8_t* const sinkp = a.part + (long long)a.npd * a.part_stride;  // 256 B behind the volumes
  const rsrc_t rpart = make_rsrc(part);
  const rsrc_t rcr = make_rsrc(a.cr);
  // staged partial stores (STAGED: batched launches, where throughput counts; a lone
  // frame's horizontal lines are its longest chains, and the flush would lengthen them): on
  // lines whose consecutive pixels are consecutive in memory (horizontal), a fast chunk
  // collects its 16 steps' bytes in LDS (16 x 16 per group), then lane j writes pixel
  // t0 + j's slot group (16 or 12 bytes, or 8 bytes of six-bit slots) with one store: whole
  // cache lines, one store instruction per chunk instead of one per step
  __shared__ uint8_t stage_tile[4 * 64 * 16];
  const bool hstage = STAGED && LPL == 16 && OUT == OUT_PART &&
                      (a.capP == 16 || a.capP == 12 || a.capP == PART6_PITCH) && (la.dp == 1 || la.dp == -1);
  // six-bit slots (levels with one line per lane whose energies fit six bits): a lane's byte
  // cannot be stored alone, so every chunk goes through the tile, fast or not
  const bool p6 = hstage && a.capP == PART6_PITCH;
  // lanes past the slot pitch keep their bytes (every band fits the first capP slots): the
  // 12-slot layout of batched levels with one line per lane, whose lane groups hold only the
  // horizontal lines (staged in fast chunks, so only the per-step stores check)
  const bool slot_ok = j < a.capP;
  uint8_t* const tile = stage_tile + (threadIdx.x & ~15) * 16;  // this group's 16 x 16 bytes

  uint32_t ring[PREFETCH];  // right census of this lane's candidate
  uint32_t bw[PREFETCH];    // broadcast step words (left census | band start << 24)
  int bl[PREFETCH];         // broadcast band lengths
  // Right census of candidate d = b0 + j at census offset c: the census margin (at least
  // D + 64 words left of x = 0) keeps c - b0 - j in bounds for every lane (b0 <= D-1).
  // For 64-lane groups c and b0 are wave-uniform: scalar base, constant lane offset.
  const uint32_t loff = (uint32_t)(LPL - 1 - j) << 2;
  // SRC_MERGE: this lane's slot of both source volumes (low and high half), loaded
  // PREFETCH steps ahead; off and uni as in the full-range scan.
  const rsrc_t rmA = make_rsrc(src_merge(SRC) ? a.msrc : a.part);
  const rsrc_t rmB = make_rsrc(src_merge(SRC) ? a.msrc + a.part_stride : a.part);
  uint32_t mring[PREFETCH];
  auto fetch_m = [&](uint32_t off, bool uni) -> uint32_t {
    if constexpr (src_merge(SRC)) {
      const uint32_t vo = uni ? (uint32_t)j : off + j, so = uni ? off : 0u;
      return buf_ld8(rmA, vo, so) | (buf_ld8(rmB, vo, so) << 16);
    } else {
      return 0u;
    }
  };
  auto fetch_c = [&](uint32_t c, uint32_t w) -> uint32_t {
    if constexpr (src_census(SRC)) {
      const uint32_t b0 = w >> 24;
      if constexpr (LPL == 64)
        return buf_ld32(rcr, loff, (c - b0 - (uint32_t)(LPL - 1)) << 2);
      else
        return buf_ld32(rcr, (c - b0 - (uint32_t)j) << 2, 0u);
    } else {
      return 0u;
    }
  };
  uint2 cur = load_chunk<true, SRC>(a, la, 0, kk);
  static_for<PREFETCH>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    bw[q] = (uint32_t)group_bcast<LPL, q>((int)cur.x);
    if constexpr (BL) bl[q] = group_bcast<LPL, q>((int)cur.y);
    ring[q] = fetch_c(la.cen(q), bw[q]);
    mring[q] = fetch_m(la.pix(q) * (uint32_t)a.capP, false);
  });
  const uint32_t pstep = (uint32_t)(la.dp * a.capP);

  // One step; FAST as in the full-range scan (no clamps, no border test, no sink).
  auto step = [&](auto kc, auto fc, const uint2& nxt, int t0, uint32_t pst, uint32_t cpf, auto stc) {
    constexpr int k = decltype(kc)::value;
    constexpr bool FAST = decltype(fc)::value;
    constexpr bool STAGE = decltype(stc)::value;
    constexpr int slot = k % PREFETCH;
    const int t = t0 + k;
    const uint32_t w = bw[slot];
    const int b0 = (int)(w >> 24);
    const int bn = VAR ? (GRAD ? bl[slot] & 0xFFFF : bl[slot]) : a.cap;
    // transition weight of this step: lambda, or the edge's gradient weight (eq. EU)
    const int lam_s = GRAD ? (int)((uint32_t)bl[slot] >> 16) : a.lambda;
    const uint32_t lt_s = GRAD ? (uint32_t)(lam_s * a.tau) : lt;
    const int lam_up = occ ? 2 * lam_s : lam_s;
    const uint32_t crv = ring[slot];
    const uint32_t mv = mring[slot];
    {  // step t + PREFETCH: broadcast its word and issue its census (or source) loads
      constexpr int kn = (k + PREFETCH) % CHUNK;
      const uint2 src = k + PREFETCH < CHUNK ? cur : nxt;
      const uint32_t wn = (uint32_t)group_bcast<LPL, kn>((int)src.x);
      if constexpr (BL) bl[slot] = group_bcast<LPL, kn>((int)src.y);
      bw[slot] = wn;
      ring[slot] = fetch_c(FAST ? cpf : la.cen(t + PREFETCH), wn);
      mring[slot] = fetch_m(FAST ? pst + (uint32_t)PREFETCH * pstep
                                 : la.pix(t + PREFETCH) * (uint32_t)a.capP,
                            FAST && LPL == 64);
    }
    uint32_t C;
    if constexpr (src_census(SRC)) {
      uint32_t pc = (uint32_t)__popc((w & 0xFFFFFFu) ^ crv);
      if constexpr (!FAST) {
        const int x = la.x0 + la.tt(t) * la.dx;
        pc = (x - b0 - j >= 0) ? pc : 24u;
      }
      C = pc + ((j < bn) ? 0u : INF32);
    } else if constexpr (src_merge(SRC)) {
      const uint32_t ua = mv & 0xFFu, ub = mv >> 16;
      C = (j < bn) ? (a.mop == MERGE_MEAN ? (ua + ub) >> 1 : min(ua, ub)) : INF32;
    } else {
      C = (j < bn) ? (uint32_t)a.cost[(size_t)la.pix(t) * a.cap + min(j, a.cap - 1)] : INF32;
    }
    uint32_t L, m, sb;
    const int src = j + (b0 - lo_prev) + e;
    if constexpr (TAU > 0) {
      // complement encoding: Pu = INF32 - P (absent 0), larger is better
      int E = band_envelope_c<LPL, TAU>(Pu, lam_s, lam_up);  // lane i <-> position i - e
      if constexpr (src_occ(SRC)) {
        if (occ) E = max(E, suffix_max_lanes<LPL>(zshift_up<LPL, TAU - 1>(Pu)) - (int)lt_s);
      }
      // batched launches: a source outside the group reads the group's last lane instead, whose
      // envelope is absent (0): its position lies more than tau-1 slots past every band slot,
      // since the host keeps cap + 2(tau-1) < LPL (the layered merge's occlusion term is not
      // absent there). Single-frame launches keep the select, which schedules their latency-bound
      // chains better.
      int Ev;
      if constexpr (src_occ(SRC) || !STAGED) {
        const int got = __builtin_amdgcn_ds_bpermute((gbase + (src & (LPL - 1))) << 2, E);
        Ev = ((unsigned)src < (unsigned)LPL) ? got : 0;
      } else {
        Ev = __builtin_amdgcn_ds_bpermute((gbase + (int)min((unsigned)src, (unsigned)(LPL - 1))) << 2, E);
      }
      int cu = GRAD ? mprev - (int)lt_s : capu;
      if constexpr (src_occ(SRC)) {
        if (occ) {
          if (src < 0) Ev = cu;  // every node of p-r lies at least tau above d
          cu -= (int)lt_s;       // increases of tau or more cost 2*lambda*tau
        }
      }
      // (the fast chunks of batched launches never hold a line's first pixel)
      const int Mu = (FAST && STAGED) || t != 0 ? max(Ev, cu) : (int)INF32;
      // a slot past the band (cost INF32 and up) is absent: batched launches leave it at
      // Mu - C <= 0, below every present value (INF32 - L > 0) in each maximum that follows;
      // the others set it to 0
      const int Lu = (STAGED && !src_occ(SRC)) || j < bn ? Mu - (int)C : 0;
      Pu = Lu;  // next state
      int mu;
      if constexpr (LPL == 64)
        mu = wave_max_s(Lu);
      else
        mu = group_max<LPL>(Lu);
      capu = mu - (int)lt;
      if constexpr (GRAD) mprev = mu;
      L = (j < bn) ? INF32 - (uint32_t)Lu : INF32;  // canonical energy itself
      m = 0;                                          // (no offset to carry)
      P = (j < bn) ? (uint32_t)(mu - Lu) : INF32;    // energy minus the line minimum
      sb = (uint32_t)(mu - Lu);  // its byte where the slot is in the band, else unused
    } else {
      uint32_t E = band_envelope<LPL, TAU>(P, a.tau, lam_s, lam_up);  // lane i <-> position i - e
      if constexpr (src_occ(SRC)) {
        if (occ) E = min(E, suffix_min_lanes<LPL>(shift_up<LPL>(P, a.tau - 1, INF32), INF32) + lt_s);
      }
      const uint32_t got =
          (uint32_t)__builtin_amdgcn_ds_bpermute((gbase + (src & (LPL - 1))) << 2, (int)E);
      uint32_t Ev = ((unsigned)src < (unsigned)LPL) ? got : INF32;
      uint32_t cl = lt_s;
      if constexpr (src_occ(SRC)) {
        if (occ) {
          if (src < 0) Ev = lt_s;  // every node of p-r lies at least tau above d
          cl = 2 * lt_s;           // increases of tau or more cost 2*lambda*tau
        }
      }
      L = C + (t == 0 ? 0u : min(Ev, cl));
      m = group_min<LPL>(L);
      P = (j < bn) ? L - m : INF32;
      sb = min(P, 255u);
    }
    if constexpr (OUT == OUT_PART) {
      const uint8_t v8 = (uint8_t)min(P, 255u);
      if constexpr (STAGE) {
        // staged slots past the band are never read (the reduce and the layered merges test
        // the band length), so the tile takes the normalised energy's byte unclamped
        tile[k * 16 + j] = (uint8_t)sb;
      } else if constexpr (FAST) {
        const uint32_t vo = LPL == 64 ? (uint32_t)j : pst + j, so = LPL == 64 ? pst : 0u;
        __builtin_amdgcn_raw_buffer_store_b8(v8, rpart, (int)vo, (int)so, 0);
      } else {
        *(t < la.n && slot_ok ? part + la.pix(t) * (uint32_t)a.capP + j : sinkp + lane) = v8;
      }
    } else {
      if (t < la.n && j < bn) export_canonical<OUT>(a.agg, (size_t)la.pix(t) * a.cap + j, L + acc, a.first);
    }
    acc += m;
    lo_prev = b0;
  };

  for (int t0 = 0; t0 < nmax; t0 += CHUNK) {
    const uint2 nxt = load_chunk<true, SRC>(a, la, t0 + CHUNK, kk);
    const int xa = la.x0 + t0 * la.dx, xb = xa + (CHUNK - 1) * la.dx;
    const bool fast = wave_all(t0 + CHUNK + PREFETCH <= la.n && (!STAGED || t0 > 0) &&
                               (!src_census(SRC) || min(xa, xb) >= a.D - 1));
    if (fast && hstage) {
      const uint32_t pst0 = (uint32_t)(la.p0 + t0 * la.dp) * (uint32_t)a.capP;
      uint32_t pst = pst0;
      uint32_t cpf = (uint32_t)(la.c0 + (t0 + PREFETCH) * la.dc);
      static_for<CHUNK>([&](auto kc) {
        step(kc, std::true_type{}, nxt, t0, pst, cpf, std::true_type{});
        pst += pstep;
        cpf += (uint32_t)la.dc;
      });
      // lane j of the group: pixel t0 + j's capP slots (offset in the vector register: see
      // the one-line-per-lane scans)
      __builtin_amdgcn_wave_barrier();
      const uint4 v = *(const uint4*)(tile + j * 16);
      const int vo = (int)(pst0 + (uint32_t)j * pstep);
      if (p6) {
        __builtin_amdgcn_raw_buffer_store_b64(pack6_bytes(v), rpart, vo, 0, kPartStorePolicy);
      } else if (a.capP == 16) {
        typedef unsigned int u4v __attribute__((ext_vector_type(4)));
        const u4v w = {v.x, v.y, v.z, v.w};
        __builtin_amdgcn_raw_buffer_store_b128(w, rpart, vo, 0, kPartStorePolicy);
      } else {
        typedef unsigned int u3v __attribute__((ext_vector_type(3)));
        const u3v w = {v.x, v.y, v.z};
        __builtin_amdgcn_raw_buffer_store_b96(w, rpart, vo, 0, kPartStorePolicy);
      }
    } else if (fast) {
      uint32_t pst = (uint32_t)(la.p0 + t0 * la.dp) * (uint32_t)a.capP;
      uint32_t cpf = (uint32_t)(la.c0 + (t0 + PREFETCH) * la.dc);
      static_for<CHUNK>([&](auto kc) {
        step(kc, std::true_type{}, nxt, t0, pst, cpf, std::false_type{});
        pst += pstep;
        cpf += (uint32_t)la.dc;
      });
    } else if (STAGED && p6) {
      if constexpr (STAGED) {
        static_for<CHUNK>([&](auto kc) { step(kc, std::false_type{}, nxt, t0, 0u, 0u, std::true_type{}); });
        __builtin_amdgcn_wave_barrier();
        const uint4 v = *(const uint4*)(tile + j * 16);
        if (t0 + j < la.n)
          __builtin_amdgcn_raw_buffer_store_b64(pack6_bytes(v), rpart, (int)(la.pix(t0 + j) * (uint32_t)PART6_PITCH),
                                                0, kPartStorePolicy);
      }
    } else {
      static_for<CHUNK>([&](auto kc) { step(kc, std::false_type{}, nxt, t0, 0u, 0u, std::false_type{}); });
    }
    cur = nxt;
  }
}

// Scan kernels: one descriptor (kernel argument) or a batch of descriptors (device table).
// Blocks hold blockDim.x / 64 independent waves; waves past the work exit at once.
// The top pyramid level's scan with the finer levels' census tiles as extra blocks: blocks
// [0, nscan) run the scan's waves, blocks nscan + v*ncen + i the census tile cen0 + i of
// view v. The top level's waves are too few to fill the chip, so the finer levels' census
// runs beside them instead of before them.
// SRC: a census source (the sum of the paths or a layered merge's first layer, with or
// without the occlusion weight and gradient weights).
template <int LPL, int K, int SRC, int TAU>
__global__ __launch_bounds__(256) void k_scan_full_cen(ScanArgs a, CenPyr cp, int nscan, int cen0,
                                                       int ncen) {
  if ((int)blockIdx.x >= nscan) {
    const int b = (int)blockIdx.x - nscan;
    census_pyr_tile(cp, cen0 + b % ncen, b / ncen);
    return;
  }
  const int u = wave_unit();
  if (u < a.gprefix[a.ndir]) scan_full_wave<LPL, K, SRC, OUT_PART, TAU, false>(a, a, u);
}

template <int LPL, int K, int SRC, int OUT, int TAU, bool BANDED>
__global__ __launch_bounds__(256) void k_scan_full(ScanArgs a) {
  const int u = wave_unit();
  if (u < a.gprefix[a.ndir]) scan_full_wave<LPL, K, SRC, OUT, TAU, BANDED>(a, a, u);
}

template <int LPL, int K, int SRC, int OUT, int TAU, bool BANDED>
__global__ __launch_bounds__(256) void k_scan_full_batch(Batch<ScanArgs> b) {
  const int u = wave_unit();
  if (u >= b.first[b.nseg]) return;
  const int s = batch_find(b.first, b.nseg, u);
  // a private copy: read once (scalar loads), not re-read after every partial store
  const ScanArgs a = b.desc[s];
  scan_full_wave<LPL, K, SRC, OUT, TAU, BANDED>(a, b.desc[s], u - b.first[s]);
}

template <int LPL, int SRC, int OUT, int TAU, bool VAR>
__global__ __launch_bounds__(256) void k_scan_band(ScanArgs a) {
  const int u = wave_unit();
  if (u < a.gprefix[a.ndir]) scan_band_wave<LPL, SRC, OUT, TAU, VAR>(a, a, u);
}

template <int LPL, int SRC, int OUT, int TAU, bool VAR>
__global__ __launch_bounds__(256) void k_scan_band_batch(Batch<ScanArgs> b) {
  const int u = wave_unit();
  if (u >= b.first[b.nseg]) return;
  const int s = batch_find(b.first, b.nseg, u);
  const ScanArgs a = b.desc[s];  // private copy, as above
  scan_band_wave<LPL, SRC, OUT, TAU, VAR, true>(a, b.desc[s], u - b.first[s]);
}

// ---------------------------------------------------------------------------------------
// Sum of paths + winner-take-all + right disparity + LR check. One block per image row.
// ---------------------------------------------------------------------------------------






// Sum of the P normalised partials of SPL consecutive slots starting at q (SPL in {1,2,4}).
// Every partial is <= 255 and P <= 8, so the 16-bit lanes of a packed sum never carry.
template <int SPL>
__device__ __forceinline__ void sum_partials(const uint8_t* q, long long stride, int np,
                                             uint32_t (&v)[SPL]) {
  if constexpr (SPL == 1) {
    uint32_t s = 0;
    for (int r = 0; r < np; ++r) s += q[r * stride];
    v[0] = s;
  } else if constexpr (SPL == 2) {
    uint32_t s = 0;
    for (int r = 0; r < np; ++r) {
      const uint32_t w = *(const uint16_t*)(q + r * stride);
      s += (w & 0xFFu) | ((w & 0xFF00u) << 8);
    }
    v[0] = s & 0xFFFFu;
    v[1] = s >> 16;
  } else {
    uint32_t e = 0, o = 0;
    for (int r = 0; r < np; ++r) {
      const uint32_t w = *(const uint32_t*)(q + r * stride);
      e += w & 0x00FF00FFu;
      o += (w >> 8) & 0x00FF00FFu;
    }
    v[0] = e & 0xFFFFu;
    v[1] = o & 0xFFFFu;
    v[2] = e >> 16;
    v[3] = o >> 16;
  }
}

// Right-disparity key: smaller S' first, then the larger disparity (the nearer surface).
__device__ __forceinline__ unsigned long long rkey(uint32_t sp, int d) {
  return ((unsigned long long)sp << 9) | (unsigned long long)(511 - d);
}
constexpr unsigned long long NOKEY = ~0ull;

template <int LPP, int SPL, int IN>
__global__ __launch_bounds__(256) void k_reduce(RedArgs a) {
  __shared__ unsigned long long s_rkey[RED_MAXW];
  __shared__ int16_t s_dl[RED_MAXW];
  const int y = blockIdx.x;
  const int tid = threadIdx.x;
  for (int x = tid; x < a.W; x += 256) s_rkey[x] = NOKEY;
  __syncthreads();
  const int lane = lane_id();
  const int wave = tid >> 6;
  const int jl = lane % LPP;
  const int pg = lane / LPP;
  constexpr int PPW = 64 / LPP;  // pixels per wave step
  const int xsteps = (a.W + 4 * PPW - 1) / (4 * PPW);
  for (int it = 0; it < xsteps; ++it) {
    const int x = (it * 4 + wave) * PPW + pg;
    const bool xin = x < a.W;
    const size_t p = (size_t)y * a.W + (xin ? x : a.W - 1);
    int b0, bn;
    band_at(a.lo, a.len, p, a.D, a.bcap, b0, bn);
    const int j0 = jl * SPL;
    uint32_t v[SPL];
    if constexpr (IN == IN_PART) {
      if (j0 < a.stride) {
        sum_partials<SPL>(a.part + p * a.stride + j0, a.part_stride, a.npart, v);
      } else {
#pragma unroll
        for (int s = 0; s < SPL; ++s) v[s] = 0;
      }
    } else {
#pragma unroll
      for (int s = 0; s < SPL; ++s) {
        const int jj = j0 + s;
        v[s] = 0;
        if (jj < a.stride) {
          if constexpr (IN == IN_U16)
            v[s] = ((const uint16_t*)a.agg)[p * a.stride + jj];
          else
            v[s] = (uint32_t)((const int32_t*)a.agg)[p * a.stride + jj];
        }
      }
    }
    bool valid[SPL];
    uint32_t vmin = 0xFFFFFFFFu;
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      const int jj = j0 + s;
      valid[s] = jj < a.stride && (a.absolute ? (jj >= b0 && jj < b0 + bn) : jj < bn);
      if (valid[s]) vmin = min(vmin, v[s]);
    }
    const uint32_t ms = group_min<LPP>(vmin);
    uint32_t jb = 0xFFFFu;
#pragma unroll
    for (int s = 0; s < SPL; ++s)
      if (valid[s] && v[s] == ms) jb = min(jb, (uint32_t)(j0 + s));
    const int jstar = (int)group_min<LPP>(jb);
    const int dl = a.absolute ? jstar : b0 + jstar;
    if (xin) {
      if (jl == 0) {
        s_dl[x] = (int16_t)dl;
        if (a.raw) a.raw[p] = (int16_t)dl;
      }
#pragma unroll
      for (int s = 0; s < SPL; ++s) {
        if (!valid[s]) continue;
        const int d = a.absolute ? j0 + s : b0 + j0 + s;
        const int xr = x - d;
        if (xr >= 0) atomicMin(&s_rkey[xr], rkey(v[s] - ms, d));
      }
    }
  }
  __syncthreads();
  for (int x = tid; x < a.W; x += 256) {
    const size_t p = (size_t)y * a.W + x;
    const unsigned long long k = s_rkey[x];
    if (a.right) a.right[p] = k == NOKEY ? (int16_t)-1 : (int16_t)(511 - (int)(k & 511ull));
    const int dl = s_dl[x];
    int16_t o = (int16_t)dl;
    if (a.lr >= 0) {
      o = -1;
      if (x - dl >= 0) {
        const unsigned long long kr = s_rkey[x - dl];
        if (kr != NOKEY) {
          const int dr = 511 - (int)(kr & 511ull);
          if (abs(dl - dr) <= a.lr) o = (int16_t)dl;
        }
      }
    }
    if (a.disp) a.disp[p] = o;
  }
}

// Fused-path reduce over the P uint8 partial volumes (their sum, or for a layered merge
// the smaller or the floor mean of the last layer's two): a lane owns SL = 16 consecutive
// slots of one pixel (one 16-byte load per partial), LPP = stride/16 lanes per pixel, 64/LPP
// pixels per wave step; or (stride 12, the compact layout of the one-line-per-lane scans)
// SL = 12 slots, one lane per pixel. Sums fit 16 bits (P * 255), so two slots share a
// register. SL = PART6_SLOTS: the six-bit layout (8 bytes per pixel, one lane per pixel), whose
// sums fit 9 bits: fields 12 bits apart share a register. need_lr = false (intermediate
// pyramid levels) writes the raw winner only.
template <int LPP, int SL = 16>
__device__ __forceinline__ void reduce_part_row(const RedArgs& a, int y, int need_lr) {
  constexpr bool P6 = SL == PART6_SLOTS;
  static_assert(SL == 16 || ((SL == 12 || P6) && LPP == 1),
                "16-slot lanes, or one 12-slot or six-bit lane per pixel");
  constexpr int NQ = P6 ? 2 : SL / 4;  // 32-bit words of slots per lane
  __shared__ uint32_t s_rkey[RED_MAXW];
  __shared__ int16_t s_dl[RED_MAXW];
  constexpr uint32_t NOK = 0xFFFFFFFFu;
  const int tid = threadIdx.x, nt = blockDim.x, nw = nt >> 6;
  if (need_lr) {
    for (int x = tid; x < a.W; x += nt) s_rkey[x] = NOK;
    __syncthreads();
  }
  const int lane = lane_id();
  const int wave = tid >> 6;
  const int jl = lane % LPP;
  const int j0 = jl * SL;
  constexpr int PPW = 64 / LPP;  // pixels per wave step
  const int xsteps = (a.W + nw * PPW - 1) / (nw * PPW);
  for (int it = 0; it < xsteps; ++it) {
    const int x = (it * nw + wave) * PPW + lane / LPP;
    const bool xin = x < a.W;
    const size_t p = (size_t)y * a.W + (xin ? x : a.W - 1);
    // every direction's slots are loaded before any is used (npart <= 8, uniform); the
    // partial volumes are read once, so the loads are non-temporal
    const uint8_t* q0 = a.part + p * a.stride + j0;
    uint32_t wv[8][NQ];
    typedef unsigned int vq __attribute__((ext_vector_type(NQ)));
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      vq w = {};
      if (r < a.npart) w = __builtin_nontemporal_load((const vq*)(q0 + r * a.part_stride));
#pragma unroll
      for (int q = 0; q < NQ; ++q) wv[r][q] = w[q];
    }
    int b0, bn;
    band_at(a.lo, a.len, p, a.D, a.bcap, b0, bn);
    // s[2q]: slots 4q (lo), 4q+2 (hi); s[2q+1]: slots 4q+1 (lo), 4q+3 (hi)
    uint32_t sm[2 * NQ];
#pragma unroll
    for (int i = 0; i < 2 * NQ; ++i) sm[i] = 0;
    uint32_t v[SL];
    if constexpr (P6) {
      // the sum of the paths (the layout serves no layered merge): word q's fields 5q, 5q+2
      // at bits 0, 12 of sm[2q], 5q+1, 5q+3 at bits 0, 12 of sm[2q+1], fields 4 and 9 at bits
      // 0 and 12 of s4
      uint32_t s4 = 0;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          sm[2 * q] += wv[r][q] & 0x3F03Fu;
          sm[2 * q + 1] += (wv[r][q] >> 6) & 0x3F03Fu;
        }
        s4 += (wv[r][0] >> 24) | ((wv[r][1] >> 12) & 0x3F000u);
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        v[5 * q + 0] = sm[2 * q] & 0xFFFu;
        v[5 * q + 1] = sm[2 * q + 1] & 0xFFFu;
        v[5 * q + 2] = sm[2 * q] >> 12;
        v[5 * q + 3] = sm[2 * q + 1] >> 12;
      }
      v[4] = s4 & 0xFFFu;
      v[9] = s4 >> 12;
    } else {
      if (a.merge == 1 + MERGE_MIN) {  // layered merge: the smaller of the two passes
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          sm[2 * q] = pk_min(wv[0][q] & 0x00FF00FFu, wv[1][q] & 0x00FF00FFu);
          sm[2 * q + 1] = pk_min((wv[0][q] >> 8) & 0x00FF00FFu, (wv[1][q] >> 8) & 0x00FF00FFu);
        }
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            sm[2 * q] += wv[r][q] & 0x00FF00FFu;
            sm[2 * q + 1] += (wv[r][q] >> 8) & 0x00FF00FFu;
          }
        }
        if (a.merge == 1 + MERGE_MEAN)  // layered merge: the mean of the two, rounded down
#pragma unroll
          for (int i = 0; i < 2 * NQ; ++i) sm[i] = (sm[i] >> 1) & 0x7FFF7FFFu;
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        v[4 * q + 0] = sm[2 * q] & 0xFFFFu;
        v[4 * q + 1] = sm[2 * q + 1] & 0xFFFFu;
        v[4 * q + 2] = sm[2 * q] >> 16;
        v[4 * q + 3] = sm[2 * q + 1] >> 16;
      }
    }
    uint32_t best = NOK;
#pragma unroll
    for (int i = 0; i < SL; ++i) {
      const int jj = j0 + i;
      const bool ok = a.absolute ? (jj >= b0 && jj < b0 + bn) : jj < bn;
      best = min(best, ok ? (v[i] << 9) | (uint32_t)jj : NOK);
    }
    best = small_group_min<LPP>(best);
    const uint32_t ms = best >> 9;
    const int jstar = (int)(best & 511u);
    const int dl = a.absolute ? jstar : b0 + jstar;
    if (xin) {
      if (jl == 0) {
        if (a.raw) a.raw[p] = (int16_t)dl;
        if (need_lr) s_dl[x] = (int16_t)dl;
        if (a.nlo) {  // the 2x2 finer pixels of this one, and the odd last column / row
          const int16_t v = (int16_t)min(max(2 * dl - a.nR, 0), a.nD - a.ncap);
          const int fx1 = x == a.W - 1 ? a.nW : min(2 * x + 2, a.nW);
          const int fy1 = y == a.H - 1 ? a.nH : min(2 * y + 2, a.nH);
          for (int fy = 2 * y; fy < fy1; ++fy)
            for (int fx = 2 * x; fx < fx1; ++fx) a.nlo[(size_t)fy * a.nW + fx] = v;
        }
      }
      if (need_lr) {
#pragma unroll
        for (int i = 0; i < SL; ++i) {
          const int jj = j0 + i;
          const bool ok = a.absolute ? (jj >= b0 && jj < b0 + bn) : jj < bn;
          const int d = a.absolute ? jj : b0 + jj;
          if (ok && x - d >= 0) atomicMin(&s_rkey[x - d], ((v[i] - ms) << 9) | (uint32_t)(511 - d));
        }
      }
    }
  }
  if (!need_lr) return;
  __syncthreads();
  for (int x = tid; x < a.W; x += nt) {
    const size_t p = (size_t)y * a.W + x;
    const uint32_t k = s_rkey[x];
    if (a.right) a.right[p] = k == NOK ? (int16_t)-1 : (int16_t)(511 - (int)(k & 511u));
    const int dl = s_dl[x];
    int16_t o = (int16_t)dl;
    if (a.lr >= 0) {
      o = -1;
      if (x - dl >= 0) {
        const uint32_t kr = s_rkey[x - dl];
        if (kr != NOK && abs(dl - (511 - (int)(kr & 511u))) <= a.lr) o = (int16_t)dl;
      }
    }
    if (a.disp) a.disp[p] = o;
  }
}

// Blocks of 256 threads, or 1024 for pixels of 4 or more lanes (more loads in flight per row).
template <int LPP, int SL = 16>
__global__ __launch_bounds__(1024) void k_reduce_part(RedArgs a, int need_lr) {
  reduce_part_row<LPP, SL>(a, blockIdx.x, need_lr);
}

// Batched: one block per image row of every pair; need_lr is per descriptor (a.lr_need).
template <int LPP, int SL = 16>
__global__ __launch_bounds__(1024) void k_reduce_part_batch(Batch<RedArgs> b) {
  const int u = blockIdx.x;
  const int s = batch_find(b.first, b.nseg, u);
  const RedArgs a = b.desc[s];  // private copy: not re-read after every store
  reduce_part_row<LPP, SL>(a, u - b.first[s], a.need_lr);
}




// ---------------------------------------------------------------------------------------
// Batched per-pixel stages: a descriptor per pair, 64x4-pixel tiles, both views per pair.
// ---------------------------------------------------------------------------------------


__device__ __forceinline__ bool batch_pixel(const Batch<PixArgs>& b, const PixArgs*& a, int& view,
                                            int& x, int& y) {
  const int u = blockIdx.x;
  const int s = batch_find(b.first, b.nseg, u);
  a = &b.desc[s];
  int t = u - b.first[s];
  view = t >= a->tiles;
  t -= view * a->tiles;
  x = (t % a->tiles_x) * 64 + (threadIdx.x & 63);
  y = (t / a->tiles_x) * 4 + (threadIdx.x >> 6);
  return x < a->W && y < a->H;
}

#ifdef MPV_MISC_KERNELS
// One 64 x CENSUS_TILE_ROWS census tile per block: the tile and its 2-pixel border
// (coordinates clamped to the image, as the census clamps its neighbours) are read into LDS
// once, then every thread takes one column of the tile, comparing each pixel with its 24
// neighbours there. Tall tiles amortise the block's descriptor lookup.
__global__ __launch_bounds__(256) void k_census_batch(Batch<PixArgs> b) {
  constexpr int R = CENSUS_TILE_ROWS;
  __shared__ uint8_t tile[R + 4][68];
  const int u = blockIdx.x;
  const int s = batch_find(b.first, b.nseg, u);
  const PixArgs* a = &b.desc[s];
  int t = u - b.first[s];
  const int v = t >= a->tiles;
  t -= v * a->tiles;
  const int W = a->W, H = a->H;
  const int x0 = (t % a->tiles_x) * 64, y0 = (t / a->tiles_x) * R;
  const uint8_t* img = a->in[v];
  const int pitch = a->in_pitch[v];
  for (int i = threadIdx.x; i < (R + 4) * 68; i += 256) {
    const int ty = i / 68, tx = i - ty * 68;
    const int x = min(max(x0 + tx - 2, 0), W - 1), y = min(max(y0 + ty - 2, 0), H - 1);
    tile[ty][tx] = img[(size_t)y * pitch + x];
  }
  __syncthreads();
  const int tx = threadIdx.x & 63;
  const int x = x0 + tx;
  if (x >= W) return;
  uint32_t* const out = (uint32_t*)a->out[v] + a->omargin + x;
#pragma unroll
  for (int r = 0; r < R / 4; ++r) {
    const int ty = (threadIdx.x >> 6) + 4 * r;
    const int y = y0 + ty;
    if (y >= H) break;
    const int c = tile[ty + 2][tx + 2];
    uint32_t val = 0;
    int bit = 0;
#pragma unroll
    for (int dy = -2; dy <= 2; ++dy)
#pragma unroll
      for (int dx = -2; dx <= 2; ++dx) {
        if (dx == 0 && dy == 0) continue;
        val |= (uint32_t)(tile[ty + 2 + dy][tx + 2 + dx] < c) << bit;
        ++bit;
      }
    out[(size_t)y * a->opitch] = val;
  }
}
#endif


#ifdef MPV_MISC_KERNELS
__global__ __launch_bounds__(256) void k_downsample_batch(Batch<PixArgs> b) {
  const PixArgs* a;
  int v, x, y;
  if (!batch_pixel(b, a, v, x, y)) return;
  const uint8_t* r0 = a->in[v] + (size_t)(2 * y) * a->in_pitch[v] + 2 * x;
  const uint8_t* r1 = r0 + a->in_pitch[v];
  ((uint8_t*)a->out[v])[(size_t)y * a->W + x] = (uint8_t)((r0[0] + r0[1] + r1[0] + r1[1] + 2) >> 2);
}
#endif





template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ p, size_t n, T v) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    p[i] = v;
}

}  // namespace mpvk
