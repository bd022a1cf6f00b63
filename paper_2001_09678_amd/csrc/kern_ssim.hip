// SSIM data term (Section 3.2, eqs. components and ssim) as a uint8 cost volume [H][W][cap].
//
// With the cited similarity index's constants (C1 = (0.01*255)^2, C2 = (0.03*255)^2,
// C3 = C2/2, unit exponents) the product of luminance, contrast and structure is exactly
//   SSIM = (2 mu_psi mu_phi + C1)(2 cov + C2) / ((mu_psi^2 + mu_phi^2 + C1)(var_psi + var_phi + C2))
// for 5x5 patches with uniform weights. In patch sums over n = 25 pixels (A, B of each patch,
// AA, BB of their squares, AB of the products) and scaled by n^2 * 10^4 every factor is an
// integer below 2^40, so SSIM = F / G with F = f1*f2, G = g1*g2 exactly in 128-bit integers,
// and the cost (1 - SSIM) * 24 / 2 rounded half up is the largest k in 0..24 with
// 24 F <= (25 - 2k) G (a 5-step search over k, no division).
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "launch.hpp"

namespace mpvk {

constexpr int SSIM_TX = 64;  // output columns per workgroup (one row)

__device__ __forceinline__ int ssim_cost_q(long long A, long long B, long long AA, long long BB,
                                           long long AB) {
  constexpr long long n2 = 625;
  const long long f1 = 20000 * A * B + 65025 * n2;                      // 2 mu mu' + C1
  const long long f2 = 20000 * (25 * AB - A * B) + 585225 * n2;         // 2 cov + C2
  const long long g1 = 10000 * (A * A + B * B) + 65025 * n2;            // mu^2 + mu'^2 + C1
  const long long g2 = 10000 * (25 * (AA + BB) - A * A - B * B) + 585225 * n2;  // var + var' + C2
  const __int128 F24 = (__int128)24 * ((__int128)f1 * f2);
  const __int128 G = (__int128)g1 * g2;
  int lo = 0, hi = 24;  // k = 0 always qualifies: F <= G
#pragma unroll
  for (int it = 0; it < 5; ++it) {
    const int k = (lo + hi + 1) >> 1;
    if (F24 <= (__int128)(25 - 2 * k) * G)
      lo = k;
    else
      hi = k - 1;
  }
  return lo;
}

// blockIdx.x: 64-column tile, blockIdx.y: row. LDS: the five rows y-2..y+2 (clamped) of the
// left image over the tile's columns +-2, of the right image over every candidate column
// (x - d for d < D) +-2, and the patch sums of each column of both.
__global__ __launch_bounds__(256) void k_cost_ssim(const uint8_t* __restrict__ L, int lpitch,
                                                   const uint8_t* __restrict__ R, int rpitch, int W,
                                                   int H, const int16_t* __restrict__ lo,
                                                   const uint8_t* __restrict__ len, int cap, int D,
                                                   uint8_t* __restrict__ cost) {
  extern __shared__ int s_ssim[];
  const int y = blockIdx.y, x0 = blockIdx.x * SSIM_TX;
  const int LW = SSIM_TX + 4;      // left tile columns x0-2 .. x0+TX+1
  const int RN = SSIM_TX + D;      // right patch centres u = x0-D .. x0+TX-1
  const int RW = RN + 4;           // right tile columns x0-D-2 .. x0+TX+1
  int* sA = s_ssim;                // [TX] left patch sums
  int* sAA = sA + SSIM_TX;         // [TX] left sums of squares
  int* sB = sAA + SSIM_TX;         // [RN] right patch sums
  int* sBB = sB + RN;              // [RN]
  uint8_t* lt = (uint8_t*)(sBB + RN);  // [5][LW]
  uint8_t* rt = lt + 5 * LW;           // [5][RW]
  const int t = threadIdx.x;
  for (int i = t; i < 5 * LW; i += 256) {
    const int r = i / LW, c = i % LW;
    lt[i] = L[(size_t)min(max(y - 2 + r, 0), H - 1) * lpitch + min(max(x0 - 2 + c, 0), W - 1)];
  }
  for (int i = t; i < 5 * RW; i += 256) {
    const int r = i / RW, c = i % RW;
    rt[i] = R[(size_t)min(max(y - 2 + r, 0), H - 1) * rpitch + min(max(x0 - D - 2 + c, 0), W - 1)];
  }
  __syncthreads();
  for (int i = t; i < SSIM_TX; i += 256) {
    int a = 0, aa = 0;
    for (int r = 0; r < 5; ++r)
      for (int c = 0; c < 5; ++c) {
        const int v = lt[r * LW + i + c];
        a += v;
        aa += v * v;
      }
    sA[i] = a;
    sAA[i] = aa;
  }
  for (int i = t; i < RN; i += 256) {
    int b = 0, bb = 0;
    for (int r = 0; r < 5; ++r)
      for (int c = 0; c < 5; ++c) {
        const int v = rt[r * RW + i + c];
        b += v;
        bb += v * v;
      }
    sB[i] = b;
    sBB[i] = bb;
  }
  __syncthreads();
  // node n of the tile: column x0 + n / cap, slot n % cap (the tile's bytes are contiguous)
  const int nx = min(SSIM_TX, W - x0), nodes = nx * cap;
  uint8_t* out = cost + ((size_t)y * W + x0) * cap;
  for (int n = t; n < nodes; n += 256) {
    const int xl = n / cap, j = n % cap, x = x0 + xl;
    int b0, bn;
    band_at(lo, len, (size_t)y * W + x, D, cap, b0, bn);
    uint8_t c = 0xFF;
    if (j < bn) {
      const int d = b0 + j;
      if (x - d < 0) {
        c = 24;
      } else {
        const int i = xl + D - d;  // right patch centre x - d, relative to x0 - D
        int ab = 0;
        for (int r = 0; r < 5; ++r)
          for (int k = 0; k < 5; ++k) ab += (int)lt[r * LW + xl + k] * (int)rt[r * RW + i + k];
        c = (uint8_t)ssim_cost_q(sA[xl], sB[i], sAA[xl], sBB[i], ab);
      }
    }
    out[n] = c;
  }
}

}  // namespace mpvk

namespace mpvl {

void cost_ssim(const uint8_t* L, int lpitch, const uint8_t* R, int rpitch, int W, int H,
               const int16_t* lo, const uint8_t* len, int cap, int D, uint8_t* cost, hipStream_t s) {
  using mpvk::SSIM_TX;
  const size_t lds = (size_t)(2 * SSIM_TX + 2 * (SSIM_TX + D)) * sizeof(int) + 5 * (SSIM_TX + 4) +
                     5 * (SSIM_TX + D + 4);
  hipLaunchKernelGGL(mpvk::k_cost_ssim, dim3((W + SSIM_TX - 1) / SSIM_TX, H), dim3(256), lds, s, L, lpitch,
                     R, rpitch, W, H, lo, len, cap, D, cost);
}

}  // namespace mpvl
