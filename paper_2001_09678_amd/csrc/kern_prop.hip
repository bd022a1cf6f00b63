// Search bands of a finer pyramid level in the paper's own form (Section 3.4): the pixels
// sampled from the coarser level carry twice its raw winner; an intermediate level takes
// the mode of those values per block, the last level interpolates linearly between them.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace mpvk {

// One 64-thread workgroup per block of the finer level. The block's parents (the coarser
// pixels (min(x/2, Wc-1), min(y/2, Hc-1)) of its pixels, a contiguous rectangle) are counted
// into an LDS histogram of raw disparities; the mode is the largest key count*512 + (511 - v),
// i.e. the most frequent value, the smallest on ties. Every pixel of the block gets the band
// start of twice the mode.
__global__ __launch_bounds__(64) void k_prop_block(PropArgs a) {
  __shared__ int hist[256];
  const int x0 = blockIdx.x * a.block, y0 = blockIdx.y * a.block;
  const int x1 = min(x0 + a.block, a.W), y1 = min(y0 + a.block, a.H);
  const int cx0 = min(x0 / 2, a.Wc - 1), cx1 = min((x1 - 1) / 2, a.Wc - 1);
  const int cy0 = min(y0 / 2, a.Hc - 1), cy1 = min((y1 - 1) / 2, a.Hc - 1);
  const int t = threadIdx.x;
  for (int i = t; i < 256; i += 64) hist[i] = 0;
  __syncthreads();
  const int nx = cx1 - cx0 + 1, n = nx * (cy1 - cy0 + 1);
  for (int k = t; k < n; k += 64) {
    const int v = a.raw[(size_t)(cy0 + k / nx) * a.Wc + cx0 + k % nx];
    atomicAdd(&hist[min(max(v, 0), 255)], 1);
  }
  __syncthreads();
  int best = 0;
  for (int v = t; v < 256; v += 64) best = max(best, hist[v] * 512 + (511 - v));
  for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o));
  const int mode = 511 - (best & 511);
  const int16_t lo = (int16_t)min(max(2 * mode - a.R, 0), a.D - a.cap);
  const int w = x1 - x0, npx = w * (y1 - y0);
  for (int k = t; k < npx; k += 64) a.lo[(size_t)(y0 + k / w) * a.W + x0 + k % w] = lo;
}

// One thread per pixel of the last level: the (up to) four samples around the pixel, each
// twice a coarser raw winner, averaged with rounding half up (exact for the samples
// themselves and for the midpoints between two).
__global__ __launch_bounds__(256) void k_prop_interp(PropArgs a) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= a.W || y >= a.H) return;
  const int i0 = min(x >> 1, a.Wc - 1), i1 = min((x >> 1) + (x & 1), a.Wc - 1);
  const int j0 = min(y >> 1, a.Hc - 1), j1 = min((y >> 1) + (y & 1), a.Hc - 1);
  const int16_t* r0 = a.raw + (size_t)j0 * a.Wc;
  const int16_t* r1 = a.raw + (size_t)j1 * a.Wc;
  const int s = 2 * ((int)r0[i0] + (int)r0[i1] + (int)r1[i0] + (int)r1[i1]);
  const int c = (s + 2) >> 2;
  a.lo[(size_t)y * a.W + x] = (int16_t)min(max(c - a.R, 0), a.D - a.cap);
}

}  // namespace mpvk

namespace mpvl {

void propagate(const PropArgs& a, hipStream_t s) {
  if (a.block > 0)
    hipLaunchKernelGGL(mpvk::k_prop_block, dim3((a.W + a.block - 1) / a.block, (a.H + a.block - 1) / a.block),
                       dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(mpvk::k_prop_interp, dim3((a.W + 63) / 64, (a.H + 3) / 4), dim3(256), 0, s, a);
}

}  // namespace mpvl
