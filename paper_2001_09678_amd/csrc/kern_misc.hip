// Per-pixel kernels (census, the all-level census of a pyramid, downsample, cost export,
// fill) and the reduce kernels (which also write the next level's band).
#define MPV_MISC_KERNELS
#include "kernels.hpp"
#include "launch.hpp"

namespace mpvl {
using namespace mpvk;

namespace {
dim3 pix_grid(int W, int H, int views) {
  return dim3((W + 63) / 64, (H + 3) / 4, views);
}
}  // namespace

void reduce_part(const RedArgs& a, int need_lr, hipStream_t s) {
  if (a.stride == 12) {
    hipLaunchKernelGGL((k_reduce_part<1, 12>), dim3(a.H), dim3(256), 0, s, a, need_lr);
    return;
  }
  switch (a.stride / 16) {
    case 1: hipLaunchKernelGGL(k_reduce_part<1>, dim3(a.H), dim3(256), 0, s, a, need_lr); break;
    case 2: hipLaunchKernelGGL(k_reduce_part<2>, dim3(a.H), dim3(256), 0, s, a, need_lr); break;
    case 4: hipLaunchKernelGGL(k_reduce_part<4>, dim3(a.H), dim3(1024), 0, s, a, need_lr); break;
    case 8: hipLaunchKernelGGL(k_reduce_part<8>, dim3(a.H), dim3(1024), 0, s, a, need_lr); break;
    default: hipLaunchKernelGGL(k_reduce_part<16>, dim3(a.H), dim3(1024), 0, s, a, need_lr); break;
  }
}

void reduce_part_batch(const Batch<RedArgs>& b, int rows, int stride, hipStream_t s) {
  if (stride == PART6_PITCH) {
    hipLaunchKernelGGL((k_reduce_part_batch<1, PART6_SLOTS>), dim3(rows), dim3(256), 0, s, b);
    return;
  }
  if (stride == 12) {
    hipLaunchKernelGGL((k_reduce_part_batch<1, 12>), dim3(rows), dim3(256), 0, s, b);
    return;
  }
  switch (stride / 16) {
    case 1: hipLaunchKernelGGL(k_reduce_part_batch<1>, dim3(rows), dim3(256), 0, s, b); break;
    case 2: hipLaunchKernelGGL(k_reduce_part_batch<2>, dim3(rows), dim3(256), 0, s, b); break;
    case 4: hipLaunchKernelGGL(k_reduce_part_batch<4>, dim3(rows), dim3(1024), 0, s, b); break;
    case 8: hipLaunchKernelGGL(k_reduce_part_batch<8>, dim3(rows), dim3(1024), 0, s, b); break;
    default: hipLaunchKernelGGL(k_reduce_part_batch<16>, dim3(rows), dim3(1024), 0, s, b); break;
  }
}

template <int IN>
static void reduce_in(const RedArgs& a, hipStream_t s) {
  const int st = a.stride;
  if (st <= 16)
    hipLaunchKernelGGL((k_reduce<16, 1, IN>), dim3(a.H), dim3(256), 0, s, a);
  else if (st <= 32)
    hipLaunchKernelGGL((k_reduce<32, 1, IN>), dim3(a.H), dim3(256), 0, s, a);
  else if (st <= 64)
    hipLaunchKernelGGL((k_reduce<64, 1, IN>), dim3(a.H), dim3(256), 0, s, a);
  else if (st <= 128)
    hipLaunchKernelGGL((k_reduce<64, 2, IN>), dim3(a.H), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_reduce<64, 4, IN>), dim3(a.H), dim3(256), 0, s, a);
}

void reduce_agg(const RedArgs& a, int in, hipStream_t s) {
  if (in == IN_U16)
    reduce_in<IN_U16>(a, s);
  else
    reduce_in<IN_I32>(a, s);
}

void census(const uint8_t* L, int lpitch, const uint8_t* R, int rpitch, int W, int H,
            uint32_t* cl, uint32_t* cr, int opitch, int omargin, hipStream_t s) {
  hipLaunchKernelGGL(k_census, pix_grid(W, H, R ? 2 : 1), dim3(256), 0, s, L, W, H, lpitch, cl,
                     opitch, omargin, R ? R : L, R ? rpitch : lpitch, R ? cr : cl);
}

void downsample(const uint8_t* in, int pitch, uint8_t* out, const uint8_t* in2, int pitch2,
                uint8_t* out2, int w, int h, hipStream_t s) {
  hipLaunchKernelGGL(k_downsample, pix_grid(w, h, in2 ? 2 : 1), dim3(256), 0, s, in, pitch, out, w,
                     h, in2 ? in2 : in, in2 ? pitch2 : pitch, in2 ? out2 : out);
}

void cost(const uint8_t* L, int lpitch, const uint8_t* R, int rpitch, int W, int H,
          const int16_t* lo, const uint8_t* len, int cap, int D, uint8_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_cost, dim3(H), dim3(256), 2 * W * sizeof(uint32_t), s, L, lpitch, R, rpitch,
                     W, H, lo, len, cap, D, out);
}

void census_pyr(const CenPyr& cp, hipStream_t s, int nblocks) {
  hipLaunchKernelGGL(k_census_pyr, dim3(nblocks < 0 ? cp.first[cp.L] : nblocks, 2), dim3(256), 0, s, cp);
}

void fill_u16(uint16_t* p, size_t n, uint16_t v, hipStream_t s) {
  const int b = (int)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill<uint16_t>, dim3(b), dim3(256), 0, s, p, n, v);
}

void fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t s) {
  const int b = (int)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(b), dim3(256), 0, s, p, n, v);
}

void census_batch(const Batch<PixArgs>& b, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_census_batch, dim3(blocks), dim3(256), 0, s, b);
}

void downsample_batch(const Batch<PixArgs>& b, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_downsample_batch, dim3(blocks), dim3(256), 0, s, b);
}

}  // namespace mpvl
