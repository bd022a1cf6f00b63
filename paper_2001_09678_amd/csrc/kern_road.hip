// Road profile in v-disparity space (Section 3.5): the v-disparity image of a disparity
// map (eq. disp_map), its column-wise counterpart (eq. hy) and the max-sum road path over
// the former (eqs. P_hat and e).
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace mpvk {

// One block per image row: an LDS histogram of the row's disparities, then column j of
// the [D][H] v-disparity image. Invalid (-1) and out-of-range disparities are not counted.
__global__ __launch_bounds__(256) void k_vdisparity(const int16_t* __restrict__ disp, int W, int H,
                                                    int pitch, int D, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int j = blockIdx.x;
  for (int i = threadIdx.x; i < D; i += 256) h[i] = 0;
  __syncthreads();
  const int16_t* row = disp + (size_t)j * pitch;
  for (int x = threadIdx.x; x < W; x += 256) {
    const int d = row[x];
    if (d >= 0 && d < D) atomicAdd(&h[d], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < D; i += 256) hist[(size_t)i * H + j] = h[i];
}

// One block per tile of COLS image columns: a wave reads 64 / COLS rows of the tile, the
// 16 waves take every (1024 / COLS)-th row, and the counts gather in an LDS histogram
// [D][COLS]; then columns j0 .. j0+COLS-1 of each disparity's line of the [D][W]
// u-disparity image. Invalid (-1) and out-of-range disparities are not counted.
constexpr int UDISP_THREADS = 1024;
template <int COLS>
__global__ __launch_bounds__(UDISP_THREADS) void k_udisparity(const int16_t* __restrict__ disp, int W,
                                                              int H, int pitch, int D,
                                                              uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256 * COLS];
  const int c = threadIdx.x % COLS;
  const int rg = threadIdx.x / COLS;
  const int x = blockIdx.x * COLS + c;
  for (int k = threadIdx.x; k < D * COLS; k += UDISP_THREADS) h[k] = 0;
  __syncthreads();
  if (x < W) {
    const int16_t* col = disp + x;
#pragma unroll 4
    for (int y = rg; y < H; y += UDISP_THREADS / COLS) {
      const int d = col[(size_t)y * pitch];
      if (d >= 0 && d < D) atomicAdd(&h[d * COLS + c], 1u);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < D * COLS; k += UDISP_THREADS) {
    const int xo = blockIdx.x * COLS + k % COLS;
    if (xo < W) hist[(size_t)(k / COLS) * W + xo] = h[k];
  }
}

// One block: disparity steps i = 1 .. D-1 in turn, each row j a node whose predecessors
// are the rows j-eta+1 .. j-1 of step i-1 (energies ping-pong in LDS, -1 = unreachable).
// back[i][j] keeps j minus the chosen predecessor (the smallest row among the maxima); the
// end is the smallest row maximising the last step, traced back by one thread. The counts
// of CHUNK steps are loaded together ahead of their use (so one load latency covers CHUNK
// dependent steps); LDS_BACK keeps the back-pointers in dynamic LDS (D*H bytes), else
// they go to the caller's workspace. Each energy row has ROAD_PAD leading entries that stay
// -1 (rows above the image: never a predecessor). NARROW (eta <= ROAD_PAD + 1): the window
// lies within the ROAD_PAD entries before row j, read without range checks and masked at
// its lower edge by a test uniform over the block; the step is bound by instruction issue
// on the one CU, so this is what sets its speed. Otherwise the window is read in groups of
// 8 with per-row range checks.
constexpr int ROAD_PAD = 8;

template <bool LDS_BACK, bool NARROW, int THREADS, int RPT, int CHUNK>
__global__ __launch_bounds__(THREADS) void k_road(const uint32_t* __restrict__ hist, int D, int H, int eta,
                                                  uint8_t* __restrict__ gback, int16_t* __restrict__ path,
                                                  int32_t* __restrict__ energy) {
  __shared__ int e[2][ROAD_PAD + ROAD_MAX_HEIGHT];
  __shared__ unsigned long long s_key[THREADS / 64];
  extern __shared__ uint8_t lback[];
  uint8_t* back = LDS_BACK ? lback : gback;
  const int tid = threadIdx.x;
  if (tid < 2 * ROAD_PAD) e[tid / ROAD_PAD][tid % ROAD_PAD] = -1;
  for (int j = tid; j < H; j += THREADS) e[0][ROAD_PAD + j] = (int)hist[j];
  __syncthreads();
  for (int i0 = 1; i0 < D; i0 += CHUNK) {
    uint32_t hv[CHUNK][RPT];
#pragma unroll
    for (int s = 0; s < CHUNK; ++s)
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int j = tid + r * THREADS;
        hv[s][r] = (i0 + s < D && j < H) ? hist[(size_t)(i0 + s) * H + j] : 0u;
      }
#pragma unroll
    for (int s = 0; s < CHUNK; ++s) {
      const int i = i0 + s;
      if (i < D) {  // uniform over the block
        const int* ep = e[(i - 1) & 1] + ROAD_PAD;
        int* ec = e[i & 1] + ROAD_PAD;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
          const int j = tid + r * THREADS;
          if (j < H) {
            int best = -1, arg = j;
            if (NARROW) {
              // entries j-8 .. j-1 (the padding above row 0 reads -1); those below j-eta+1
              // masked; maximum and first maximising entry in ascending row order (strictly
              // greater: the smallest row wins ties; -1 entries never win)
              int v[ROAD_PAD];
#pragma unroll
              for (int k = 0; k < ROAD_PAD; ++k) v[k] = ep[j - ROAD_PAD + k];
#pragma unroll
              for (int k = 0; k < ROAD_PAD; ++k)
                if (k < ROAD_PAD + 1 - eta) v[k] = -1;
              int bk = ROAD_PAD;
#pragma unroll
              for (int k = 0; k < ROAD_PAD; ++k) {
                bk = v[k] > best ? k : bk;
                best = v[k] > best ? v[k] : best;
              }
              arg = j - ROAD_PAD + bk;
            } else {
              for (int base = j - eta + 1; base < j; base += 8) {
                int v[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                  const int jp = base + k;
                  v[k] = (jp >= 0 && jp < j) ? ep[jp] : -1;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k)
                  if (v[k] > best) {
                    best = v[k];
                    arg = base + k;
                  }
              }
            }
            ec[j] = best >= 0 ? (int)hv[s][r] + best : -1;
            back[(size_t)i * H + j] = (uint8_t)(j - arg);
          }
        }
        __syncthreads();
      }
    }
  }
  // end of the profile: maximum energy, smallest row on ties (key = energy, then ~row)
  const int* el = e[(D - 1) & 1] + ROAD_PAD;
  unsigned long long key = 0;
  for (int j = tid; j < H; j += THREADS)
    if (el[j] >= 0) {
      const unsigned long long k = ((unsigned long long)(unsigned)el[j] << 32) | (0xFFFFFFFFu - (unsigned)j);
      key = k > key ? k : key;
    }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(key, o);
    key = other > key ? other : key;
  }
  if ((tid & 63) == 0) s_key[tid >> 6] = key;
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < THREADS / 64; ++w) key = s_key[w] > key ? s_key[w] : key;
    if (key == 0) {  // nothing reachable at the last disparity
      for (int i = 0; i < D; ++i) path[i] = -1;
      *energy = -1;
    } else {
      int j = (int)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFu));
      *energy = (int32_t)(key >> 32);
      path[D - 1] = (int16_t)j;
      for (int i = D - 1; i > 0; --i) {
        j -= back[(size_t)i * H + j];
        path[i - 1] = (int16_t)j;
      }
    }
  }
}

}  // namespace mpvk

namespace mpvl {
using namespace mpvk;

void vdisparity(const int16_t* disp, int W, int H, int pitch, int D, uint32_t* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_vdisparity, dim3(H), dim3(256), 0, s, disp, W, H, pitch, D, hist);
}

template <int COLS>
void udisparity_cols(const int16_t* disp, int W, int H, int pitch, int D, uint32_t* hist, hipStream_t s) {
  hipLaunchKernelGGL(k_udisparity<COLS>, dim3((W + COLS - 1) / COLS), dim3(UDISP_THREADS), 0, s, disp, W,
                     H, pitch, D, hist);
}

// 16-column tiles: a 1280-wide map gets 80 workgroups. Measured at 1280x720 (D=128), 640x360
// (D=64) and 1920x1080 (D=256), 16 columns take 3.8, 3.4 and 5.1 us per launch against
// 9.2, 5.5 and 13.4 us for 64-column tiles (too few workgroups) and within 0.4 us of 8.
void udisparity(const int16_t* disp, int W, int H, int pitch, int D, uint32_t* hist, hipStream_t s) {
  udisparity_cols<16>(disp, W, H, pitch, D, hist, s);
}

// Back-pointers in LDS up to this many bytes (beside the 32 KB of energies).
constexpr size_t ROAD_LDS_BACK = 96 * 1024;

// One shape of the road workgroup: THREADS threads own RPT rows each (THREADS * RPT >= H)
// and prefetch the counts of CHUNK steps (CHUNK * RPT registers).
template <bool NARROW, int THREADS, int RPT, int CHUNK>
void road_cfg(const uint32_t* hist, int D, int H, int eta, uint8_t* back, int16_t* path, int32_t* energy,
              hipStream_t s) {
  static_assert(THREADS * RPT <= ROAD_MAX_HEIGHT && THREADS % 64 == 0 && THREADS >= 2 * ROAD_PAD,
                "road workgroup shape");
  const size_t bytes = (size_t)D * H;
  static const bool lds_ok =
      hipFuncSetAttribute((const void*)k_road<true, NARROW, THREADS, RPT, CHUNK>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)ROAD_LDS_BACK) == hipSuccess;
  if (lds_ok && bytes <= ROAD_LDS_BACK)
    hipLaunchKernelGGL((k_road<true, NARROW, THREADS, RPT, CHUNK>), dim3(1), dim3(THREADS), bytes, s, hist, D,
                       H, eta, back, path, energy);
  else
    hipLaunchKernelGGL((k_road<false, NARROW, THREADS, RPT, CHUNK>), dim3(1), dim3(THREADS), 0, s, hist, D, H,
                       eta, back, path, energy);
}

// 1024 threads with as few rows each as the height allows: rows a thread does not own
// still cost it branches at every step, and the step is bound by instruction issue. At
// 720 rows (D = 128, eta = 8) one row per thread takes 51 us against 67 us with four; at
// 1080 rows (D = 256) two take 174 us against 201 us.
template <bool NARROW>
void road_rows(const uint32_t* hist, int D, int H, int eta, uint8_t* back, int16_t* path, int32_t* energy,
               hipStream_t s) {
  if (H <= 1024)
    road_cfg<NARROW, 1024, 1, 16>(hist, D, H, eta, back, path, energy, s);
  else if (H <= 2048)
    road_cfg<NARROW, 1024, 2, 16>(hist, D, H, eta, back, path, energy, s);
  else
    road_cfg<NARROW, 1024, 4, 16>(hist, D, H, eta, back, path, energy, s);
}

void road(const uint32_t* hist, int D, int H, int eta, uint8_t* back, int16_t* path, int32_t* energy,
          hipStream_t s) {
  if (eta <= ROAD_PAD + 1)
    road_rows<true>(hist, D, H, eta, back, path, energy, s);
  else
    road_rows<false>(hist, D, H, eta, back, path, energy, s);
}

}  // namespace mpvl
