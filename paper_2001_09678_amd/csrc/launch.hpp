// Host-callable launchers. Every kernel template is instantiated in exactly one
// translation unit (kern_*.hip); the API code (mpv.hip) only calls these functions.
#pragma once
#include <hip/hip_runtime.h>

#include "types.hpp"

namespace mpvl {
using mpvk::Batch;
using mpvk::CenPyr;
using mpvk::PixArgs;
using mpvk::PropArgs;
using mpvk::RedArgs;
using mpvk::ScanArgs;

// Full-range scan layouts (lanes per line, packed pairs per lane) with kernels.
bool full_layout_ok(int LPL, int K);

// Scans. `a.tau` is the reduced tau; fused partial-output scans (SRC_CENSUS, OUT_PART)
// have compile-time versions for tau 1, 2 and 4, everything else uses runtime tau.
// wpb = waves per block (1, 2 or 4).
void scan_full(const ScanArgs& a, int LPL, int K, int src, int out, bool banded, int wpb,
               hipStream_t s);
void scan_full_batch(const Batch<ScanArgs>& b, int units, int LPL, int K, int tau, bool banded,
                     int wpb, hipStream_t s);
void scan_band(const ScanArgs& a, int LPL, int src, int out, bool var, int wpb, hipStream_t s);
void scan_band_batch(const Batch<ScanArgs>& b, int units, int LPL, int tau, int wpb, hipStream_t s);
// One line per lane for the directions with dy != 0 (kern_band_lines.hip): band lengths and
// reduced tau with kernels, then a batch of descriptors whose directions all have dy != 0
// (ScanArgs::line_lanes, gprefix counting 64 lines per wave), 12 partial slots per pixel, or
// (p6) six-bit slots in PART6_PITCH bytes.
bool band_line_ok(int cap, int tau);
void scan_lane_batch(const Batch<ScanArgs>& b, int units, int cap, int tau, bool p6, int wpb,
                     hipStream_t s);
// Cost-volume source with partial output (the fused SSIM path; kern_cost_src.hip).
void scan_full_cost(const ScanArgs& a, int LPL, int K, bool banded, int wpb, hipStream_t s);
void scan_band_cost(const ScanArgs& a, int LPL, bool var, int wpb, hipStream_t s);
// Unfused export (SRC_COST, OUT_U16 / OUT_I32) of the full-range scans.
void scan_full_export(const ScanArgs& a, int LPL, int K, int out, bool banded, int wpb, hipStream_t s);
// Layered path merge: src = SRC_MERGE (later layers: the merge of the previous layer's
// partials a.msrc, a.mop) or SRC_CENSUS_OCC (first layer with the occlusion weight on
// a.up_dir); partial output; tau 1, 2, 4 compile-time, others runtime.
void scan_full_layered(const ScanArgs& a, int src, int LPL, int K, bool banded, int wpb,
                       hipStream_t s);
void scan_band_layered(const ScanArgs& a, int src, int LPL, bool var, int wpb, hipStream_t s);
void scan_full_batch_layered(const Batch<ScanArgs>& b, int src, int units, int LPL, int K, int tau,
                             bool banded, int wpb, hipStream_t s);
// The occlusion-weight source of the layered full-range scans (units of their own).
void scan_full_occ(const ScanArgs& a, int LPL, int K, bool banded, int wpb, hipStream_t s);
void scan_full_batch_occ(const Batch<ScanArgs>& b, int units, int LPL, int K, int tau, bool banded,
                         int wpb, hipStream_t s);
void scan_band_batch_layered(const Batch<ScanArgs>& b, int src, int units, int LPL, int tau, int wpb,
                             hipStream_t s);
// Gradient-weighted transitions (src includes SRC_GRAD; base SRC_CENSUS, SRC_CENSUS_OCC or
// SRC_MERGE): single-descriptor launches.
void scan_full_grad(const ScanArgs& a, int src, int LPL, int K, bool banded, int wpb, hipStream_t s);
void scan_band_grad(const ScanArgs& a, int src, int LPL, bool var, int wpb, hipStream_t s);
// Units of their own behind scan_full_grad / scan_band_grad.
void scan_full_grad_occ(const ScanArgs& a, int LPL, int K, bool banded, int wpb, hipStream_t s);
void scan_full_grad_merge(const ScanArgs& a, int LPL, int K, bool banded, int wpb, hipStream_t s);
void scan_band_grad_merge(const ScanArgs& a, int LPL, bool var, int wpb, hipStream_t s);
// Batched launches with gradient-weighted transitions (src includes SRC_GRAD).
void scan_full_batch_grad(const Batch<ScanArgs>& b, int src, int units, int LPL, int K, int tau,
                          bool banded, int wpb, hipStream_t s);
void scan_full_batch_grad_layered(const Batch<ScanArgs>& b, int src, int units, int LPL, int K, int tau,
                                  bool banded, int wpb, hipStream_t s);
void scan_band_batch_grad(const Batch<ScanArgs>& b, int src, int units, int LPL, int tau, int wpb,
                          hipStream_t s);

// Sum + WTA (+ right disparity + LR when need_lr) over P partial volumes (uint8 slots; batched:
// also six-bit slots at stride PART6_PITCH).
void reduce_part(const RedArgs& a, int need_lr, hipStream_t s);
void reduce_part_batch(const Batch<RedArgs>& b, int rows, int stride, hipStream_t s);
// WTA + right disparity + LR over an exported uint16 / int32 aggregate volume.
void reduce_agg(const RedArgs& a, int in, hipStream_t s);

// Census of one or two views (R == nullptr: one view).
void census(const uint8_t* L, int lpitch, const uint8_t* R, int rpitch, int W, int H,
            uint32_t* cl, uint32_t* cr, int opitch, int omargin, hipStream_t s);
// 2x2 downsample of one or two views to w x h (in2 == nullptr: one view).
void downsample(const uint8_t* in, int pitch, uint8_t* out, const uint8_t* in2, int pitch2,
                uint8_t* out2, int w, int h, hipStream_t s);
void cost(const uint8_t* L, int lpitch, const uint8_t* R, int rpitch, int W, int H,
          const int16_t* lo, const uint8_t* len, int cap, int D, uint8_t* cost, hipStream_t s);
// SSIM cost volume (kern_ssim.hip), same layout and band rules as cost().
void cost_ssim(const uint8_t* L, int lpitch, const uint8_t* R, int rpitch, int W, int H,
               const int16_t* lo, const uint8_t* len, int cap, int D, uint8_t* cost, hipStream_t s);
// Census tiles [0, nblocks) of every view (nblocks < 0: every level).
void census_pyr(const CenPyr& cp, hipStream_t s, int nblocks = -1);
// Top-level full-range scan (census source src: SRC_CENSUS or SRC_CENSUS_OCC, optionally
// | SRC_GRAD; partial output) with census tiles [cen0, cen0 + ncen) of both views as extra
// blocks of the launch.
void scan_full_cen(const ScanArgs& a, int src, const CenPyr& cp, int cen0, int ncen, int LPL, int K,
                   int wpb, hipStream_t s);
void scan_full_cen_grad(const ScanArgs& a, int src, const CenPyr& cp, int cen0, int ncen, int LPL, int K,
                        int wpb, hipStream_t s);
// Road profile (kern_road.hip): v-disparity image [D][H] of a disparity map, and the
// max-sum road path over it (one block; back = D*H bytes of back-pointers).
void vdisparity(const int16_t* disp, int W, int H, int pitch, int D, uint32_t* hist, hipStream_t s);
void udisparity(const int16_t* disp, int W, int H, int pitch, int D, uint32_t* hist, hipStream_t s);
void road(const uint32_t* hist, int D, int H, int eta, uint8_t* back, int16_t* path, int32_t* energy,
          hipStream_t s);
// The paper's propagation (kern_prop.hip): block modes (a.block > 0) or interpolation.
void propagate(const PropArgs& a, hipStream_t s);
void fill_u16(uint16_t* p, size_t n, uint16_t v, hipStream_t s);
void fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t s);

// Batched per-pixel stages: `blocks` = sum over descriptors of their tiles (x2 for two views).
void census_batch(const Batch<PixArgs>& b, int blocks, hipStream_t s);
void downsample_batch(const Batch<PixArgs>& b, int blocks, hipStream_t s);

// Features of a coarse level for the band-proposal network (kern_lb.hip).
void lb_features(const uint8_t* part, long long pstride, int capP, int P, int D, int W, int H,
                 const int16_t* raw, const int16_t* disp, const uint8_t* img, int ipitch, float Z,
                 uint16_t* feat, hipStream_t s);

}  // namespace mpvl
