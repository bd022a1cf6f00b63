// Argument structs shared by the kernels (device) and the launch code (host).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpvk {

// Scan sources: census (fused cost), a uint8 cost volume, the merge of the previous
// layer's two partial volumes (layered path merge), or the census with the occlusion
// weight of the layered merge (direction up_dir pays twice for disparity increases).
// SRC_GRAD (or-ed into a source): gradient-weighted transition of eq. EU, the weight of
// each edge along the line is round(lambda * exp(-|I(p) - I(p-r)| / sigma)) of the left
// image of the level.
enum { SRC_CENSUS = 0, SRC_COST = 1, SRC_MERGE = 2, SRC_CENSUS_OCC = 3, SRC_GRAD = 8 };
constexpr int src_base(int src) { return src & 7; }
constexpr bool src_grad(int src) { return (src & SRC_GRAD) != 0; }
constexpr bool src_census(int src) { return src_base(src) == SRC_CENSUS || src_base(src) == SRC_CENSUS_OCC; }
constexpr bool src_merge(int src) { return src_base(src) == SRC_MERGE; }
constexpr bool src_occ(int src) { return src_base(src) == SRC_CENSUS_OCC; }
// Merge of two partial volumes: the smaller, or the mean rounded down.
enum { MERGE_MIN = 0, MERGE_MEAN = 1 };
enum { OUT_PART = 0, OUT_U16 = 1, OUT_I32 = 2 };

struct ScanArgs {
  int W, H, D, cap;  // cap: slots per pixel of the cost volume / aggregate export
  int lambda, tau;   // tau = min(tau, D-1) clamped to >= 1 (same energies, see host)
  const uint32_t* cl;
  const uint32_t* cr;
  int cpitch, cmargin;
  const uint8_t* cost;
  const int16_t* lo;
  const uint8_t* len;
  uint8_t* part;
  long long part_stride;  // bytes between direction volumes
  int capP;               // partial slots per pixel (bytes), or PART6_PITCH: six-bit slots
  void* agg;              // canonical export [H][W][cap]
  int first;              // canonical export: this direction writes instead of adding
  // Directions of this descriptor: dir[0..ndir), their partial volumes are numbers
  // dir_base .. dir_base+ndir-1 of the pair's npd volumes; stores of steps past a line's end
  // go to a 256 B sink right after the pair's last volume.
  int ndir;
  int dir_base, npd;
  int dir[8];
  int gprefix[9];  // first wave of each direction (one wave = 64/LPL lines)
  // SRC_MERGE: the previous layer's two partial volumes, msrc and msrc + part_stride, in
  // this scan's slot layout; mop = MERGE_MIN or MERGE_MEAN.
  const uint8_t* msrc;
  int mop;
  int up_dir;  // SRC_CENSUS_OCC: the direction whose disparity increases cost 2*lambda
  // SRC_GRAD: the left image of the level ([H][ipitch]) and sigma >= 1
  const uint8_t* img;
  int ipitch, sigma;
  // 1: one line per lane (directions with dy != 0, census source, fixed-length bands);
  // gprefix then counts 64 lines per wave
  int line_lanes;
};

// Segment table of a batched launch: global wave u belongs to descriptor s with
// first[s] <= u < first[s+1] (first[] ascending, first[0] = 0).
template <typename T>
struct Batch {
  const T* desc;
  const int* first;
  int nseg;
};

enum { IN_PART = 0, IN_U16 = 1, IN_I32 = 2 };

struct RedArgs {
  int W, H, D;
  int stride;  // slots per pixel of the input volume(s)
  int bcap;    // band length where len == null (cap of the band, or D at full range)
  const int16_t* lo;
  const uint8_t* len;
  int absolute;  // slot index = absolute disparity (partials of a banded full-range scan)
  const uint8_t* part;
  long long part_stride;
  int npart;
  int merge;  // 0: sum of the npart partials; 1 + MERGE_MIN / MERGE_MEAN: of two partials
  const void* agg;
  int lr;
  int need_lr;  // batched launches: compute right disparity + LR for this descriptor
  int16_t* disp;
  int16_t* right;
  int16_t* raw;
  // Band of the next finer level (Section 3.4), written beside the raw winner: fine pixel
  // (fx, fy) takes this level's pixel (min(fx/2, W-1), min(fy/2, H-1)) and gets
  // lo = clamp(2 * raw - nR, 0, nD - ncap). Null: no finer level.
  int16_t* nlo;
  int nW, nH, nD, nR, ncap;
};

struct PixArgs {
  int W, H;                // output size of this stage
  const uint8_t* in[2];    // source images (views)
  int in_pitch[2];
  void* out[2];            // census: uint32 at y*opitch + omargin + x; downsample: uint8 [H][W]
  int opitch, omargin;
  int tiles_x, tiles;      // tiles per view
};

// Census of every pyramid level of both views in one launch (level L-1 = the input).
struct CenPyr {
  const uint8_t* img[2];  // input images (finest level)
  int pitch[2];
  int L;
  int W[4], H[4];
  uint32_t* out[4][2];  // census of level l, view v: uint32 at y*opitch + omargin + x
  uint8_t* limg[4];     // optional: the left image of level l, [H][W] (null: not written)
  int opitch[4], omargin[4];
  int tiles_x[4];
  int first[5];  // first block of each level (64x4 outputs per block)
};

// Band of a finer level from the coarser level's raw winners in the paper's own form
// (Section 3.4). block > 0 (intermediate level): every block x block tile searches around
// twice the mode of its parents' raw disparities; block == 0 (last level): sampled pixels take
// twice their parent's raw disparity, the others the linear interpolation of the samples.
// Band of every pixel: cap disparities from lo = clamp(centre - R, 0, D - cap).
struct PropArgs {
  const int16_t* raw;  // coarser level's raw winners [Hc][Wc]
  int Wc, Hc;
  int16_t* lo;  // finer level's band starts [H][W]
  int W, H, D, R, cap, block;
};

// Six-bit partial layout: a pixel's slots 0..9 in 8 bytes, slot i in bits 6*(i%5) .. +5 of
// 32-bit word i/5 (bits 30, 31 zero). Taken where every normalised energy fits six bits
// (24 + lambda*tau <= 63); the sum of 8 paths then fits 9 bits.
constexpr int PART6_PITCH = 8;
constexpr int PART6_SLOTS = 10;

constexpr int RED_MAXW = 4096;
constexpr int CENSUS_TILE_ROWS = 16;  // batched census: 64 x 16 pixels per block
constexpr int ROAD_MAX_HEIGHT = 4096;  // rows of a v-disparity image the road kernel holds in LDS

}  // namespace mpvk
