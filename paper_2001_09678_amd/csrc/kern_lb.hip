// Learned band proposal: features, BF16 MFMA convolutions (forward and backward),
// deterministic weight gradients, loss/heads, Adam, band maps (include/mpv_lb.h).
//
// Convolutions (forward and backward-data) are implicit GEMMs on gfx950's
// v_mfma_f32_16x16x32_bf16: rows = pixels (16 per wave), columns = output channels (16 per
// tile), reduction = (tap, input channel) in steps of 32. A lane holds A[pixel l%16][k
// 8*(l/16)..+7], B[k 8*(l/16)..+7][channel l%16] and receives D[pixel 4*(l/16)+i][channel
// l%16]. Input channels of a tap are contiguous in NHWC, so an A operand is one 16-byte load
// for 8 or more channels (two 8-byte loads, one per tap, for 4; zero outside the image).
// The weight gradient is a GEMM too: rows = (tap, input channel), columns = output channels,
// reduction = pixels in steps of 32 (8 gathered pixels per lane).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/mpv_lb.h"
#include "launch.hpp"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8s __attribute__((ext_vector_type(8)));    // bf16 bits, as loaded
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));    // MFMA operand type
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);  // nearest, ties to even
}
__device__ __forceinline__ float bf2f(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}
__device__ __forceinline__ bool bf_pos(uint16_t h) { return !(h & 0x8000u) && h != 0; }

constexpr int r16(int v) { return (v + 15) / 16 * 16; }
constexpr int r32(int v) { return (v + 31) / 32 * 32; }
constexpr int r4(int v) { return (v + 3) / 4 * 4; }

// ---------------------------------------------------------------------------------------
// Features of the coarse level from its P uint8 partial energy volumes.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_features(const uint8_t* __restrict__ part, long long pstride,
                                                  int capP, int P, int D, int W, int H,
                                                  const int16_t* __restrict__ raw,
                                                  const int16_t* __restrict__ disp,
                                                  const uint8_t* __restrict__ img, int ipitch,
                                                  float Z, uint16_t* __restrict__ feat) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= W * H) return;
  const int x = p % W, y = p / W;
  const uint8_t* q = part + (size_t)p * capP;
  const int dl = raw[p];
  // one sweep: global minimum, minimum over |d - dl| > 1, and S at dl-2 .. dl+2 (clamped)
  const int dm2 = max(dl - 2, 0), dm1 = max(dl - 1, 0), dp1 = min(dl + 1, D - 1), dp2 = min(dl + 2, D - 1);
  int mn = 1 << 30, far = 1 << 30, sm2 = 0, sm1 = 0, sp1 = 0, sp2 = 0;
  for (int d = 0; d < D; ++d) {
    int v = 0;
    for (int r = 0; r < P; ++r) v += q[(long long)r * pstride + d];
    mn = min(mn, v);
    if (abs(d - dl) > 1) far = min(far, v);
    if (d == dm2) sm2 = v;
    if (d == dm1) sm1 = v;
    if (d == dp1) sp1 = v;
    if (d == dp2) sp2 = v;
  }
  uint16_t* f = feat + (size_t)p * 8;
  f[0] = f2bf((float)img[(size_t)y * ipitch + x] / 255.0f);
  f[1] = f2bf((float)dl / (float)D);
  f[2] = f2bf(disp[p] >= 0 ? 1.0f : 0.0f);
  f[3] = f2bf((float)(sm1 - mn) / Z);
  f[4] = f2bf((float)(sp1 - mn) / Z);
  f[5] = f2bf((float)(sm2 - mn) / Z);
  f[6] = f2bf((float)(sp2 - mn) / Z);
  f[7] = f2bf(far == (1 << 30) ? 1.0f : (float)(far - mn) / Z);
}

// ---------------------------------------------------------------------------------------
// Convolution (forward, or backward-data with the mirrored packing).
// ---------------------------------------------------------------------------------------
template <int CIN, int NT>
__global__ __launch_bounds__(256) void k_conv(const uint16_t* __restrict__ x, int N, int H, int W,
                                              const uint16_t* __restrict__ wp,
                                              const float* __restrict__ bias, int cout, int relu,
                                              const uint16_t* __restrict__ mask, int mstride,
                                              void* __restrict__ y, int ystride, int yf32) {
  constexpr int KREAL = 9 * CIN;
  constexpr int KPAD = r32(KREAL);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long M = (long)N * H * W;
  const long mbase = ((long)blockIdx.x * 4 + wave) * 16;
  if (mbase >= M) return;
  const long pm = std::min(mbase + (lane & 15), M - 1);
  const int px = (int)(pm % W);
  const long t = pm / W;
  const int py = (int)(t % H);
  const long pn = t / H;
  const int kq = (lane >> 4) * 4;  // output rows 4*(l/16) .. +3
  const int k8 = (lane >> 4) * 8;  // reduction slice of this lane
  // 4 channels of tap `tap` from channel c of this lane's pixel (zero outside the image or K)
  auto tap4 = [&](int tap, int c) -> bf16x4 {
    bf16x4 v = {0, 0, 0, 0};
    if (tap < 9) {
      const int yy = py + tap / 3 - 1, xx = px + tap % 3 - 1;
      if (yy >= 0 && yy < H && xx >= 0 && xx < W) v = *(const bf16x4*)(x + ((pn * H + yy) * W + xx) * CIN + c);
    }
    return v;
  };
  f32x4 acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int k0 = 0; k0 < KPAD; k0 += 32) {
    const int k = k0 + k8;
    bf16x8s a = {0, 0, 0, 0, 0, 0, 0, 0};
    if constexpr (CIN % 8 == 0) {  // the 8 channels c .. c+7 of one tap
      const int tap = k / CIN, c = k % CIN;
      if (tap < 9) {
        const int yy = py + tap / 3 - 1, xx = px + tap % 3 - 1;
        if (yy >= 0 && yy < H && xx >= 0 && xx < W)
          a = *(const bf16x8s*)(x + ((pn * H + yy) * W + xx) * CIN + c);
      }
    } else {  // CIN == 4: taps k/4 and k/4 + 1
      const bf16x4 lo = tap4(k / 4, 0), hi = tap4(k / 4 + 1, 0);
      a = bf16x8s{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    }
    const bf16x8 av = __builtin_bit_cast(bf16x8, a);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n = nt * 16 + (lane & 15);
      const bf16x8 b = __builtin_bit_cast(bf16x8, *(const bf16x8s*)(wp + (size_t)n * KPAD + k));
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b, acc[nt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int n = nt * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long m = mbase + kq + i;
      if (m >= M || n >= ystride) continue;
      float v = 0.f;
      if (n < cout) {
        v = acc[nt][i] + (bias ? bias[n] : 0.f);
        if (relu) v = fmaxf(v, 0.f);
        if (mask && !bf_pos(mask[m * mstride + n])) v = 0.f;
      }
      if (yf32)
        ((float*)y)[m * ystride + n] = v;
      else
        ((uint16_t*)y)[m * ystride + n] = f2bf(v);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Weight gradient: dW[(tap,c)][n] = sum_p x(p + tap)[c] * dz[p][n] over a chunk of pixels per
// block (rows = (tap, c), columns = channels, reduction = pixels), then a fixed-order sum.
// ---------------------------------------------------------------------------------------
template <int CIN, int NT>
__global__ __launch_bounds__(256) void k_conv_dw(const uint16_t* __restrict__ x,
                                                 const uint16_t* __restrict__ dz, int dzs, int N,
                                                 int H, int W, int cout, int chunk,
                                                 float* __restrict__ part,
                                                 float* __restrict__ dbpart) {
  constexpr int KREAL = 9 * CIN;
  constexpr int MT = (KREAL + 15) / 16;
  constexpr int MTW = (MT + 3) / 4;  // M tiles per wave
  __shared__ float s_db[8][NT * 16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long M = (long)N * H * W;
  const long p_begin = (long)blockIdx.x * chunk;
  const long p_end = std::min(p_begin + chunk, M);
  const int kq = (lane >> 4) * 4;  // output rows 4*(l/16) .. +3
  const int k8 = (lane >> 4) * 8;  // this lane's 8 pixels of a 32-pixel reduction step
  f32x4 acc[MTW][NT];
#pragma unroll
  for (int j = 0; j < MTW; ++j)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[j][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (long p0 = p_begin; p0 < p_end; p0 += 32) {
    int qx[8], qy[8];
    long qn[8];
    bool qv[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const long p = p0 + k8 + i;
      qv[i] = p < p_end;
      const long pc = qv[i] ? p : p_begin;
      qx[i] = (int)(pc % W);
      const long t = pc / W;
      qy[i] = (int)(t % H);
      qn[i] = t / H;
    }
    bf16x8 b[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int n = nt * 16 + (lane & 15);
      bf16x8s v;
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (qv[i] && n < cout) ? (short)dz[(p0 + k8 + i) * dzs + n] : (short)0;
      b[nt] = __builtin_bit_cast(bf16x8, v);
    }
#pragma unroll
    for (int j = 0; j < MTW; ++j) {
      const int mt = wave + 4 * j;
      if (mt >= MT) break;
      const int m = mt * 16 + (lane & 15);
      bf16x8s a = {0, 0, 0, 0, 0, 0, 0, 0};
      if (m < KREAL) {
        const int tap = m / CIN, c = m % CIN;
        const int oy = tap / 3 - 1, ox = tap % 3 - 1;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int yy = qy[i] + oy, xx = qx[i] + ox;
          if (qv[i] && yy >= 0 && yy < H && xx >= 0 && xx < W)
            a[i] = (short)x[((qn[i] * H + yy) * W + xx) * CIN + c];
        }
      }
      const bf16x8 av = __builtin_bit_cast(bf16x8, a);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[j][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[nt], acc[j][nt], 0, 0, 0);
    }
  }
  float* dst = part + (size_t)blockIdx.x * (MT * 16) * (NT * 16);
#pragma unroll
  for (int j = 0; j < MTW; ++j) {
    const int mt = wave + 4 * j;
    if (mt >= MT) break;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        dst[(mt * 16 + kq + i) * (NT * 16) + nt * 16 + (lane & 15)] = acc[j][nt][i];
  }
  // bias gradient: 8 groups of 32 threads, group g sums pixels p = p_begin + g (mod 8)
  const int g = threadIdx.x >> 5, col = threadIdx.x & 31;
  if (col < NT * 16) {
    float s = 0.f;
    if (col < cout)
      for (long p = p_begin + g; p < p_end; p += 8) s += bf2f(dz[p * dzs + col]);
    s_db[g][col] = s;
  }
  __syncthreads();
  if (threadIdx.x < NT * 16) {
    float s = 0.f;
    for (int k = 0; k < 8; ++k) s += s_db[k][threadIdx.x];
    dbpart[(size_t)blockIdx.x * (NT * 16) + threadIdx.x] = s;
  }
}

__global__ __launch_bounds__(256) void k_dw_reduce(const float* __restrict__ part,
                                                   const float* __restrict__ dbpart, int nblk,
                                                   int rows, int cols, int kreal, int cout,
                                                   float* __restrict__ dw, float* __restrict__ db) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < kreal * cout) {
    const int m = i / cout, n = i % cout;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[((size_t)b * rows + m) * cols + n];
    dw[i] = s;
  }
  if (i < cout) {
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += dbpart[(size_t)b * cols + i];
    db[i] = s;
  }
}

// ---------------------------------------------------------------------------------------
// Weight packing
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ w, int cin, int cout,
                                              uint16_t* __restrict__ wf, uint16_t* __restrict__ wb) {
  const int kf = r32(9 * cin), nf = r16(cout);
  const int c4 = r4(cout), kb = r32(9 * c4), nb = r16(cin);
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (wf && i < nf * kf) {
    const int n = i / kf, k = i % kf;
    wf[i] = (n < cout && k < 9 * cin) ? f2bf(w[k * cout + n]) : (uint16_t)0;
  }
  if (wb && i < nb * kb) {
    const int ci = i / kb, k = i % kb;
    const int tapm = k / c4, co = k % c4;
    wb[i] = (ci < cin && tapm < 9 && co < cout) ? f2bf(w[((8 - tapm) * cin + ci) * cout + co])
                                                : (uint16_t)0;
  }
}

// ---------------------------------------------------------------------------------------
// Heads + loss
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ o,
                                              const int16_t* __restrict__ raw,
                                              const int16_t* __restrict__ labels, int N, int hc,
                                              int wc, int H, int W, float beta, float inv,
                                              uint16_t* __restrict__ dz, float* __restrict__ lossp) {
  __shared__ float s_loss[256];
  const int p = blockIdx.x * 256 + threadIdx.x;
  float lsum = 0.f;
  if (p < N * hc * wc) {
    const int cx = p % wc, t = p / wc, cy = t % hc, n = t / hc;
    const float o0 = o[p * 4 + 0], o1 = o[p * 4 + 1], o2 = o[p * 4 + 2];
    const float center = 4.0f * (float)raw[p] + o0;
    const float width = 2.0f + fminf(fmaxf(o1, 0.f), 14.f);
    const float conf = fminf(fmaxf(o2, 0.f), 1.f);
    float gc = 0.f, gw = 0.f, gq = 0.f;
    for (int by = 0; by < 4; ++by)
      for (int bx = 0; bx < 4; ++bx) {
        const int fy = cy * 4 + by, fx = cx * 4 + bx;
        if (fy >= H || fx >= W) continue;
        const int d = labels[((size_t)n * H + fy) * W + fx];
        if (d < 0) continue;
        const float e = center - (float)d;
        const float ae = fabsf(e);
        const float h = 2.f * ae + 2.f - width;
        const float ind = ae <= width * 0.5f ? 1.f : 0.f;
        const float q = conf - ind;
        lsum += (ae < 1.f ? 0.5f * e * e : ae - 0.5f) + fmaxf(h, 0.f) + beta * width + q * q;
        const float sgn = e > 0.f ? 1.f : (e < 0.f ? -1.f : 0.f);
        gc += (ae < 1.f ? e : sgn) + (h > 0.f ? 2.f * sgn : 0.f);
        gw += beta - (h > 0.f ? 1.f : 0.f);
        gq += 2.f * q;
      }
    dz[p * 4 + 0] = f2bf(gc * inv);
    dz[p * 4 + 1] = f2bf((o1 > 0.f && o1 < 14.f) ? gw * inv : 0.f);
    dz[p * 4 + 2] = f2bf((o2 > 0.f && o2 < 1.f) ? gq * inv : 0.f);
    dz[p * 4 + 3] = 0;
  }
  s_loss[threadIdx.x] = lsum * inv;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) s_loss[threadIdx.x] += s_loss[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) lossp[blockIdx.x] = s_loss[0];
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ g,
                                              long long n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ __launch_bounds__(256) void k_zero_i32(int* __restrict__ p) { p[0] = 0; }

__global__ __launch_bounds__(256) void k_bands(const float* __restrict__ o,
                                               const int16_t* __restrict__ raw, int wc, int hc,
                                               int W, int H, int D, float theta,
                                               int16_t* __restrict__ lo, uint8_t* __restrict__ len,
                                               int* __restrict__ nlow) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= W || y >= H) return;
  const int cx = min(x >> 2, wc - 1), cy = min(y >> 2, hc - 1);
  const int c = cy * wc + cx;
  const float center = 4.0f * (float)raw[c] + o[c * 4 + 0];
  const int ci = (int)floorf(center + 0.5f);
  int w = 2 + (int)fminf(fmaxf(floorf(o[c * 4 + 1] + 0.5f), 0.f), 14.f);
  const bool low = o[c * 4 + 2] < theta;  // clamp(conf, 0, 1) < theta for theta in (0, 1]
  if (low) w = 16;
  w = min(w, D);
  lo[(size_t)y * W + x] = (int16_t)min(max(ci - w / 2, 0), D - w);
  len[(size_t)y * W + x] = (uint8_t)w;
  if (low && x == (cx << 2) && y == (cy << 2)) atomicAdd(nlow, 1);
}

mpv_status launched() { return hipGetLastError() == hipSuccess ? MPV_OK : MPV_ERR_DEVICE; }

int dw_chunk() { return 1024; }

}  // namespace

namespace mpvl {
void lb_features(const uint8_t* part, long long pstride, int capP, int P, int D, int W, int H,
                 const int16_t* raw, const int16_t* disp, const uint8_t* img, int ipitch, float Z,
                 uint16_t* feat, hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3((W * H + 255) / 256), dim3(256), 0, s, part, pstride, capP,
                     P, D, W, H, raw, disp, img, ipitch, Z, feat);
}
}  // namespace mpvl

extern "C" {

size_t mpv_lb_packed_elems(int32_t cin, int32_t cout) {
  return (size_t)r16(cout) * r32(9 * cin);
}

size_t mpv_lb_packed_bwd_elems(int32_t cin, int32_t cout) {
  return (size_t)r16(cin) * r32(9 * r4(cout));
}

static bool lb_shape_ok(int cin, int cout) {
  const bool ci = cin == 4 || cin == 8 || cin == 32;
  return ci && cout >= 1 && cout <= 32;
}

mpv_status mpv_lb_pack(const float* w, int32_t cin, int32_t cout, uint16_t* wfwd, uint16_t* wbwd,
                       hipStream_t stream) {
  if (!w || (!wfwd && !wbwd) || cin < 1 || cin > 32 || cin % 4 || cout < 1 || cout > 32)
    return MPV_ERR_INVALID_ARG;
  const size_t n = std::max(mpv_lb_packed_elems(cin, cout), mpv_lb_packed_bwd_elems(cin, cout));
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, w, cin, cout,
                     wfwd, wbwd);
  return launched();
}

mpv_status mpv_lb_conv(const uint16_t* x, int32_t n, int32_t h, int32_t w, int32_t cin,
                       const uint16_t* wpacked, const float* bias, int32_t cout, int32_t relu,
                       const uint16_t* mask, int32_t mask_stride, void* y, int32_t y_stride,
                       int32_t y_f32, hipStream_t stream) {
  if (!x || !wpacked || !y || n < 1 || h < 1 || w < 1 || !lb_shape_ok(cin, cout) ||
      y_stride < cout || (mask && mask_stride < cout))
    return MPV_ERR_INVALID_ARG;
  const long M = (long)n * h * w;
  const dim3 grid((unsigned)((M + 63) / 64));
  const int nt = cout > 16 ? 2 : 1;
#define LB_CONV(CI, NT)                                                                      \
  hipLaunchKernelGGL((k_conv<CI, NT>), grid, dim3(256), 0, stream, x, n, h, w, wpacked, bias, \
                     cout, relu, mask, mask_stride, y, y_stride, y_f32)
  if (cin == 4)
    { if (nt == 2) { LB_CONV(4, 2); } else { LB_CONV(4, 1); } }
  else if (cin == 8)
    { if (nt == 2) { LB_CONV(8, 2); } else { LB_CONV(8, 1); } }
  else
    { if (nt == 2) { LB_CONV(32, 2); } else { LB_CONV(32, 1); } }
#undef LB_CONV
  return launched();
}

size_t mpv_lb_dw_workspace_bytes(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout) {
  if (n < 1 || h < 1 || w < 1 || !lb_shape_ok(cin, cout)) return 0;
  const long M = (long)n * h * w;
  const long nblk = (M + dw_chunk() - 1) / dw_chunk();
  const size_t rows = r16(9 * cin), cols = r16(cout);
  return (size_t)nblk * (rows * cols + cols) * sizeof(float);
}

mpv_status mpv_lb_conv_dw(const uint16_t* x, const uint16_t* dz, int32_t dz_stride, int32_t n,
                          int32_t h, int32_t w, int32_t cin, int32_t cout, float* dw, float* db,
                          void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!x || !dz || !dw || !db || dz_stride < cout) return MPV_ERR_INVALID_ARG;
  const size_t need = mpv_lb_dw_workspace_bytes(n, h, w, cin, cout);
  if (!need) return MPV_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < need) return MPV_ERR_WORKSPACE;
  const long M = (long)n * h * w;
  const int nblk = (int)((M + dw_chunk() - 1) / dw_chunk());
  const int rows = r16(9 * cin), cols = r16(cout);
  float* part = (float*)workspace;
  float* dbp = part + (size_t)nblk * rows * cols;
#define LB_DW(CI, NT)                                                                         \
  hipLaunchKernelGGL((k_conv_dw<CI, NT>), dim3(nblk), dim3(256), 0, stream, x, dz, dz_stride, n, \
                     h, w, cout, dw_chunk(), part, dbp)
  const int nt = cout > 16 ? 2 : 1;
  if (cin == 4)
    { if (nt == 2) { LB_DW(4, 2); } else { LB_DW(4, 1); } }
  else if (cin == 8)
    { if (nt == 2) { LB_DW(8, 2); } else { LB_DW(8, 1); } }
  else
    { if (nt == 2) { LB_DW(32, 2); } else { LB_DW(32, 1); } }
#undef LB_DW
  const int total = 9 * cin * cout;
  hipLaunchKernelGGL(k_dw_reduce, dim3((total + 255) / 256), dim3(256), 0, stream, part, dbp, nblk,
                     rows, cols, 9 * cin, cout, dw, db);
  return launched();
}

mpv_status mpv_lb_loss(const float* o, const int16_t* raw0, const int16_t* labels, int32_t n,
                       int32_t hc, int32_t wc, int32_t H, int32_t W, float beta, float inv_count,
                       uint16_t* dz, float* loss_partials, hipStream_t stream) {
  if (!o || !raw0 || !labels || !dz || !loss_partials || n < 1 || hc < 1 || wc < 1 || H < 1 ||
      W < 1)
    return MPV_ERR_INVALID_ARG;
  const int P = n * hc * wc;
  hipLaunchKernelGGL(k_loss, dim3((P + 255) / 256), dim3(256), 0, stream, o, raw0, labels, n, hc,
                     wc, H, W, beta, inv_count, dz, loss_partials);
  return launched();
}

mpv_status mpv_lb_adam(float* p, float* m, float* v, const float* g, int64_t count, float lr,
                       float beta1, float beta2, float eps, int32_t step, hipStream_t stream) {
  if (!p || !m || !v || !g || count < 1 || step < 1) return MPV_ERR_INVALID_ARG;
  const float c1 = 1.0f / (1.0f - std::pow(beta1, (float)step));
  const float c2 = 1.0f / (1.0f - std::pow(beta2, (float)step));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, p, m, v,
                     g, (long long)count, lr, beta1, beta2, eps, c1, c2);
  return launched();
}

mpv_status mpv_lb_bands(const float* o, const int16_t* raw0, int32_t wc, int32_t hc, int32_t W,
                        int32_t H, int32_t D, float theta, int16_t* lo, uint8_t* len,
                        int32_t* n_low, hipStream_t stream) {
  if (!o || !raw0 || !lo || !len || !n_low || wc < 1 || hc < 1 || W < 1 || H < 1 || D < 2 ||
      !(theta > 0.f && theta <= 1.f))
    return MPV_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, stream, n_low);
  hipLaunchKernelGGL(k_bands, dim3((W + 63) / 64, (H + 3) / 4), dim3(256), 0, stream, o, raw0, wc,
                     hc, W, H, D, theta, lo, len, n_low);
  return launched();
}

}  // extern "C"
