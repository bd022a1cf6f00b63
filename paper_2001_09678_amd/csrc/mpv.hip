// C-ABI entry points of the MPV stereo library (declared in include/mpv.h).
//
// Host code only validates, sizes the caller's workspace, picks a kernel variant and
// enqueues on the caller's stream; it never allocates and never synchronises.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstring>

#include "../../include/mpv.h"
#include "kernels.hpp"

using namespace mpvk;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v, size_t a = ALIGN) { return (v + a - 1) / a * a; }

bool valid_image(const mpv_image* im) {
  return im && im->data && im->width > 0 && im->height > 0 && im->pitch >= im->width;
}

// tau reduced to the largest disparity difference that can occur; lambda*min(|d-d'|, tau)
// is unchanged and the truncation candidate never undercuts a real predecessor.
int tau_eff(int tau, int D) { return std::max(1, std::min(tau, D - 1)); }

mpv_status check_params(const mpv_params* p, bool fused) {
  if (!p) return MPV_ERR_INVALID_ARG;
  if (p->num_disp < 1 || p->num_disp > MPV_MAX_DISP) return MPV_ERR_INVALID_ARG;
  if (p->census_radius != 2) return MPV_ERR_UNSUPPORTED;
  if (!(p->num_paths == 1 || p->num_paths == 2 || p->num_paths == 4 || p->num_paths == 8))
    return MPV_ERR_INVALID_ARG;
  if (p->lambda < 0 || p->tau < 1) return MPV_ERR_INVALID_ARG;
  const long lt = (long)p->lambda * tau_eff(p->tau, p->num_disp);
  if (fused ? (24 + lt > 255) : (lt > 4000)) return MPV_ERR_UNSUPPORTED;
  if (p->agg_type != MPV_AGG_U16 && p->agg_type != MPV_AGG_I32) return MPV_ERR_INVALID_ARG;
  return MPV_OK;
}

mpv_status check_band(const mpv_band* b, int D) {
  if (!b || !b->lo) return MPV_OK;
  if (b->cap < 1 || b->cap > D) return MPV_ERR_INVALID_ARG;
  return MPV_OK;
}

mpv_status launched() {
  return hipGetLastError() == hipSuccess ? MPV_OK : MPV_ERR_DEVICE;
}

// ---- timing hook -------------------------------------------------------------------------
struct TimingHook {
  int level = -2;  // -2: unset
  hipEvent_t before = nullptr, after = nullptr;
};
TimingHook g_hook[MPV_NUM_STAGES];

struct HookScope {  // records the stage's events around the launches made in its lifetime
  const TimingHook* h;
  hipStream_t s;
  HookScope(int stage, int level, hipStream_t st) : h(nullptr), s(st) {
    const TimingHook& t = g_hook[stage];
    if (t.before && (t.level == -1 || t.level == level)) {
      h = &t;
      (void)hipEventRecord(t.before, s);
    }
  }
  ~HookScope() {
    if (h) (void)hipEventRecord(h->after, s);
  }
};

// ---- scan layout -------------------------------------------------------------------------
struct FullLayout {
  int LPL, K;
  int dpad() const { return 2 * K * LPL; }
};
FullLayout full_layout(int D) {
  if (D <= 32) return {16, 1};
  if (D <= 64) return {32, 1};
  if (D <= 128) return {64, 1};
  return {64, 2};
}
// Smallest lane group that holds a band of `cap` plus tau-1 neighbours on each side; 0 if none.
int band_lanes(int cap, int te) {
  const int need = cap + 2 * (te - 1);
  if (need <= 16) return 16;
  if (need <= 32) return 32;
  if (need <= 64) return 64;
  return 0;
}

struct ScanChoice {
  bool banded_kernel;  // k_scan_band
  int LPL, K;
  int capP;  // partial slots per pixel
  bool absolute;
};
ScanChoice choose_scan(int D, const mpv_band* band, int tau) {
  const int te = tau_eff(tau, D);
  if (band && band->lo) {
    const int lpl = band_lanes(band->cap, te);
    if (lpl) return {true, lpl, 1, lpl, false};
    FullLayout f = full_layout(D);
    return {false, f.LPL, f.K, f.dpad(), true};
  }
  FullLayout f = full_layout(D);
  return {false, f.LPL, f.K, f.dpad(), false};
}

int num_lines_host(int r, int W, int H) {
  static const int dx[8] = {+1, -1, 0, 0, +1, -1, -1, +1};
  static const int dy[8] = {0, 0, +1, -1, +1, -1, +1, -1};
  return dy[r] == 0 ? H : (dx[r] == 0 ? W : W + H - 1);
}

// Fill direction list + block prefix; returns the number of blocks.
int plan_dirs(ScanArgs& a, const int* dirs, int ndir, int LPL) {
  a.ndir = ndir;
  int blocks = 0;
  for (int i = 0; i < ndir; ++i) {
    a.dir[i] = dirs[i];
    a.gprefix[i] = blocks;
    const int lines = num_lines_host(dirs[i], a.W, a.H);
    blocks += (lines + (64 / LPL) - 1) / (64 / LPL);
  }
  a.gprefix[ndir] = blocks;
  for (int i = ndir; i < 8; ++i) a.dir[i] = 0;
  return blocks;
}

// tau (already reduced to min(tau, D-1)) is a compile-time parameter for 1..4 on the fused
// path, so the envelope is a fixed sequence of DPP shifts; other values, and the unfused
// export path, take the runtime-tau kernels.
template <int SRC, int OUT, int TAU, bool BANDED>
void launch_full_t(const ScanArgs& a, int LPL, int K, int blocks, hipStream_t s) {
  if (LPL == 16)
    hipLaunchKernelGGL((k_scan_full<16, 1, SRC, OUT, TAU, BANDED>), dim3(blocks), dim3(64), 0, s, a);
  else if (LPL == 32)
    hipLaunchKernelGGL((k_scan_full<32, 1, SRC, OUT, TAU, BANDED>), dim3(blocks), dim3(64), 0, s, a);
  else if (K == 1)
    hipLaunchKernelGGL((k_scan_full<64, 1, SRC, OUT, TAU, BANDED>), dim3(blocks), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((k_scan_full<64, 2, SRC, OUT, TAU, BANDED>), dim3(blocks), dim3(64), 0, s, a);
}

template <int SRC, int OUT, bool BANDED>
void launch_full_b(const ScanArgs& a, int LPL, int K, int blocks, hipStream_t s) {
  if constexpr (OUT == OUT_PART) {
    switch (a.tau) {
      case 1: launch_full_t<SRC, OUT, 1, BANDED>(a, LPL, K, blocks, s); return;
      case 2: launch_full_t<SRC, OUT, 2, BANDED>(a, LPL, K, blocks, s); return;
      case 3: launch_full_t<SRC, OUT, 3, BANDED>(a, LPL, K, blocks, s); return;
      case 4: launch_full_t<SRC, OUT, 4, BANDED>(a, LPL, K, blocks, s); return;
      default: break;
    }
  }
  launch_full_t<SRC, OUT, 0, BANDED>(a, LPL, K, blocks, s);
}

template <int SRC, int OUT>
void launch_full(const ScanArgs& a, int LPL, int K, int blocks, hipStream_t s) {
  if (a.lo)
    launch_full_b<SRC, OUT, true>(a, LPL, K, blocks, s);
  else
    launch_full_b<SRC, OUT, false>(a, LPL, K, blocks, s);
}

template <int SRC, int OUT, int TAU, bool VAR>
void launch_band_v(const ScanArgs& a, int LPL, int blocks, hipStream_t s) {
  if (LPL == 16)
    hipLaunchKernelGGL((k_scan_band<16, SRC, OUT, TAU, VAR>), dim3(blocks), dim3(64), 0, s, a);
  else if (LPL == 32)
    hipLaunchKernelGGL((k_scan_band<32, SRC, OUT, TAU, VAR>), dim3(blocks), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((k_scan_band<64, SRC, OUT, TAU, VAR>), dim3(blocks), dim3(64), 0, s, a);
}

template <int SRC, int OUT, int TAU>
void launch_band_t(const ScanArgs& a, int LPL, int blocks, hipStream_t s) {
  if (a.len)
    launch_band_v<SRC, OUT, TAU, true>(a, LPL, blocks, s);
  else
    launch_band_v<SRC, OUT, TAU, false>(a, LPL, blocks, s);
}

template <int SRC, int OUT>
void launch_band(const ScanArgs& a, int LPL, int blocks, hipStream_t s) {
  if constexpr (OUT == OUT_PART) {
    switch (a.tau) {
      case 1: launch_band_t<SRC, OUT, 1>(a, LPL, blocks, s); return;
      case 2: launch_band_t<SRC, OUT, 2>(a, LPL, blocks, s); return;
      case 3: launch_band_t<SRC, OUT, 3>(a, LPL, blocks, s); return;
      case 4: launch_band_t<SRC, OUT, 4>(a, LPL, blocks, s); return;
      default: break;
    }
  }
  launch_band_t<SRC, OUT, 0>(a, LPL, blocks, s);
}

template <int IN>
void launch_reduce(const RedArgs& a, hipStream_t s) {
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

void launch_reduce_part(const RedArgs& a, int need_lr, hipStream_t s) {
  switch (a.stride / 16) {
    case 1: hipLaunchKernelGGL(k_reduce_part<1>, dim3(a.H), dim3(256), 0, s, a, need_lr); break;
    case 2: hipLaunchKernelGGL(k_reduce_part<2>, dim3(a.H), dim3(256), 0, s, a, need_lr); break;
    case 4: hipLaunchKernelGGL(k_reduce_part<4>, dim3(a.H), dim3(256), 0, s, a, need_lr); break;
    case 8: hipLaunchKernelGGL(k_reduce_part<8>, dim3(a.H), dim3(256), 0, s, a, need_lr); break;
    default: hipLaunchKernelGGL(k_reduce_part<16>, dim3(a.H), dim3(256), 0, s, a, need_lr); break;
  }
}

dim3 pix_grid(int W, int H) { return dim3((W + 63) / 64, (H + 3) / 4); }

// ---- one fused level -------------------------------------------------------------------
struct LevelWs {
  size_t census_off, part_off, total;
  int cpitch, cmargin;
  ScanChoice sc;
};

LevelWs level_ws(const mpv_params* p, int W, int H, const mpv_band* band) {
  LevelWs w{};
  w.sc = choose_scan(p->num_disp, band, p->tau);
  const int dpad = full_layout(p->num_disp).dpad();
  w.cmargin = (int)align_up((size_t)std::max(dpad, p->num_disp) + 1, 16);
  w.cpitch = w.cmargin + W;
  w.census_off = 0;
  const size_t cen = align_up((size_t)H * w.cpitch * sizeof(uint32_t));
  w.part_off = w.census_off + 2 * cen;
  // partial volumes, then a 256 B sink for stores past a line's end
  w.total = w.part_off + align_up((size_t)p->num_paths * H * W * w.sc.capP) + ALIGN;
  return w;
}

// census(L), census(R) -> all P directions -> reduce. disp may be null (intermediate level).
mpv_status run_level(const mpv_params* p, const uint8_t* L, int lpitch, const uint8_t* R,
                     int rpitch, int W, int H, const mpv_band* band, int16_t* disp,
                     int16_t* right, int16_t* raw, uint8_t* ws, int level, hipStream_t s) {
  const LevelWs lw = level_ws(p, W, H, band);
  uint32_t* cl = (uint32_t*)(ws + lw.census_off);
  uint32_t* cr = cl + align_up((size_t)H * lw.cpitch * sizeof(uint32_t)) / sizeof(uint32_t);
  uint8_t* part = ws + lw.part_off;
  {
    HookScope hs(MPV_STAGE_CENSUS, level, s);
    dim3 g = pix_grid(W, H);
    g.z = 2;
    hipLaunchKernelGGL(k_census, g, dim3(256), 0, s, L, W, H, lpitch, cl, lw.cpitch, lw.cmargin,
                       R, rpitch, cr);
  }
  ScanArgs a{};
  a.W = W;
  a.H = H;
  a.D = p->num_disp;
  a.cap = (band && band->lo) ? band->cap : p->num_disp;
  a.lambda = p->lambda;
  a.tau = tau_eff(p->tau, p->num_disp);
  a.cl = cl;
  a.cr = cr;
  a.cpitch = lw.cpitch;
  a.cmargin = lw.cmargin;
  a.lo = band ? band->lo : nullptr;
  a.len = (band && band->lo) ? band->len : nullptr;
  a.part = part;

  a.capP = lw.sc.capP;
  a.part_stride = (long long)H * W * lw.sc.capP;
  int dirs[8];
  for (int i = 0; i < p->num_paths; ++i) dirs[i] = i;
  const int blocks = plan_dirs(a, dirs, p->num_paths, lw.sc.LPL);

  {
    HookScope hs(MPV_STAGE_SCAN, level, s);
    if (lw.sc.banded_kernel)
      launch_band<SRC_CENSUS, OUT_PART>(a, lw.sc.LPL, blocks, s);
    else
      launch_full<SRC_CENSUS, OUT_PART>(a, lw.sc.LPL, lw.sc.K, blocks, s);
  }
  RedArgs ra{};
  ra.W = W;
  ra.H = H;
  ra.D = p->num_disp;
  ra.stride = lw.sc.capP;
  ra.bcap = a.cap;
  ra.lo = a.lo;
  ra.len = a.len;
  ra.absolute = lw.sc.absolute ? 1 : 0;
  ra.part = part;
  ra.part_stride = a.part_stride;
  ra.npart = p->num_paths;
  ra.lr = p->lr_max_diff;
  ra.disp = disp;
  ra.right = right;
  ra.raw = raw;
  {
    HookScope hs(MPV_STAGE_REDUCE, level, s);
    launch_reduce_part(ra, (disp || right) ? 1 : 0, s);
  }
  return launched();
}

struct PyrGeom {
  int L;
  int W[MPV_MAX_LEVELS], H[MPV_MAX_LEVELS], D[MPV_MAX_LEVELS], cap[MPV_MAX_LEVELS];
};

mpv_status pyr_geom(const mpv_pyramid_params* p, int W, int H, PyrGeom& g) {
  if (!p) return MPV_ERR_INVALID_ARG;
  mpv_status st = check_params(&p->base, true);
  if (st) return st;
  if (p->levels < 1 || p->levels > MPV_MAX_LEVELS || p->band_radius < 0) return MPV_ERR_INVALID_ARG;
  if (W < 1 || H < 1 || W > MPV_MAX_WIDTH) return MPV_ERR_INVALID_ARG;
  g.L = p->levels;
  for (int l = 0; l < g.L; ++l) {
    const int sh = g.L - 1 - l;
    g.W[l] = W >> sh;
    g.H[l] = H >> sh;
    g.D[l] = (p->base.num_disp + (1 << sh) - 1) >> sh;
    if (g.W[l] < 1 || g.H[l] < 1) return MPV_ERR_INVALID_ARG;
    g.cap[l] = l == 0 ? g.D[l] : std::min(2 * p->band_radius + 1, g.D[l]);
  }
  return MPV_OK;
}

struct PyrWs {
  size_t img_off[MPV_MAX_LEVELS];  // left at off, right at off + W*H
  size_t raw_off[MPV_MAX_LEVELS];
  size_t lo_off;
  size_t level_off;  // census + partials, reused per level
  size_t total;
};

PyrWs pyr_ws(const mpv_pyramid_params* p, const PyrGeom& g) {
  PyrWs w{};
  size_t off = 0;
  for (int l = 0; l + 1 < g.L; ++l) {
    w.img_off[l] = off;
    off += align_up((size_t)2 * g.W[l] * g.H[l]);
  }
  for (int l = 0; l < g.L; ++l) {
    w.raw_off[l] = off;
    off += align_up((size_t)g.W[l] * g.H[l] * sizeof(int16_t));
  }
  w.lo_off = off;
  off += align_up((size_t)g.W[g.L - 1] * g.H[g.L - 1] * sizeof(int16_t));
  w.level_off = off;
  size_t lvl = 0;
  for (int l = 0; l < g.L; ++l) {
    mpv_params lp = p->base;
    lp.num_disp = g.D[l];
    mpv_band b{nullptr, nullptr, g.cap[l]};
    int16_t dummy;
    if (l > 0) b.lo = &dummy;  // only presence matters for sizing
    lvl = std::max(lvl, level_ws(&lp, g.W[l], g.H[l], l > 0 ? &b : nullptr).total);
  }
  w.total = off + lvl;
  return w;
}

}  // namespace

extern "C" {

const char* mpv_status_string(mpv_status s) {
  switch (s) {
    case MPV_OK: return "MPV_OK";
    case MPV_ERR_INVALID_ARG: return "MPV_ERR_INVALID_ARG";
    case MPV_ERR_UNSUPPORTED: return "MPV_ERR_UNSUPPORTED";
    case MPV_ERR_WORKSPACE: return "MPV_ERR_WORKSPACE";
    case MPV_ERR_OVERFLOW: return "MPV_ERR_OVERFLOW";
    case MPV_ERR_DEVICE: return "MPV_ERR_DEVICE";
  }
  return "MPV_ERR_UNKNOWN";
}

mpv_status mpv_census(const mpv_image* img, uint32_t* census, hipStream_t stream) {
  if (!valid_image(img) || !census) return MPV_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_census, pix_grid(img->width, img->height), dim3(256), 0, stream, img->data,
                     img->width, img->height, img->pitch, census, img->width, 0, img->data,
                     img->pitch, census);
  return launched();
}

mpv_status mpv_downsample(const mpv_image* img, uint8_t* out, hipStream_t stream) {
  if (!valid_image(img) || !out) return MPV_ERR_INVALID_ARG;
  const int w = img->width / 2, h = img->height / 2;
  if (w < 1 || h < 1) return MPV_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_downsample, pix_grid(w, h), dim3(256), 0, stream, img->data, img->pitch,
                     out, w, h, img->data, img->pitch, out);
  return launched();
}

mpv_status mpv_cost(const mpv_params* p, const mpv_image* left, const mpv_image* right,
                    const mpv_band* band, uint8_t* cost, hipStream_t stream) {
  mpv_status st = check_params(p, false);
  if (st) return st;
  if (!valid_image(left) || !valid_image(right) || !cost) return MPV_ERR_INVALID_ARG;
  if (left->width != right->width || left->height != right->height) return MPV_ERR_INVALID_ARG;
  if ((st = check_band(band, p->num_disp))) return st;
  const int W = left->width, H = left->height;
  if (W > MPV_MAX_WIDTH) return MPV_ERR_INVALID_ARG;
  const bool banded = band && band->lo;
  const int cap = banded ? band->cap : p->num_disp;
  hipLaunchKernelGGL(k_cost, dim3(H), dim3(256), 2 * W * sizeof(uint32_t), stream, left->data,
                     left->pitch, right->data, right->pitch, W, H, banded ? band->lo : nullptr,
                     banded ? band->len : nullptr, cap, p->num_disp, cost);
  return launched();
}

mpv_status mpv_aggregate(const mpv_params* p, const uint8_t* cost, int32_t W, int32_t H,
                         const mpv_band* band, uint32_t path_mask, void* agg,
                         hipStream_t stream) {
  mpv_status st = check_params(p, false);
  if (st) return st;
  if (!cost || !agg || W < 1 || H < 1) return MPV_ERR_INVALID_ARG;
  if ((st = check_band(band, p->num_disp))) return st;
  const bool banded = band && band->lo;
  const int cap = banded ? band->cap : p->num_disp;
  int dirs[8], nd = 0;
  for (int r = 0; r < p->num_paths; ++r)
    if (!path_mask || (path_mask & (1u << r))) dirs[nd++] = r;
  if (nd == 0) return MPV_ERR_INVALID_ARG;
  const long lt = (long)p->lambda * tau_eff(p->tau, p->num_disp);
  const double bound = (double)nd * (banded ? 24 + lt : 24) * std::max(W, H);
  if (bound > (p->agg_type == MPV_AGG_U16 ? 65535.0 : 2147483647.0)) return MPV_ERR_OVERFLOW;
  const size_t n = (size_t)W * H * cap;
  const int fb = (int)std::min<size_t>((n + 255) / 256, 65536);
  if (p->agg_type == MPV_AGG_U16)
    hipLaunchKernelGGL(k_fill<uint16_t>, dim3(fb), dim3(256), 0, stream, (uint16_t*)agg, n,
                       (uint16_t)0xFFFF);
  else
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(fb), dim3(256), 0, stream, (int32_t*)agg, n,
                       (int32_t)0x7FFFFFFF);
  const ScanChoice sc = choose_scan(p->num_disp, band, p->tau);
  for (int i = 0; i < nd; ++i) {
    ScanArgs a{};
    a.W = W;
    a.H = H;
    a.D = p->num_disp;
    a.cap = cap;
    a.lambda = p->lambda;
    a.tau = tau_eff(p->tau, p->num_disp);
    a.cost = cost;
    a.lo = banded ? band->lo : nullptr;
    a.len = banded ? band->len : nullptr;
    a.agg = agg;
    a.first = i == 0;
    const int blocks = plan_dirs(a, &dirs[i], 1, sc.LPL);
    if (sc.banded_kernel) {
      if (p->agg_type == MPV_AGG_U16)
        launch_band<SRC_COST, OUT_U16>(a, sc.LPL, blocks, stream);
      else
        launch_band<SRC_COST, OUT_I32>(a, sc.LPL, blocks, stream);
    } else {
      if (p->agg_type == MPV_AGG_U16)
        launch_full<SRC_COST, OUT_U16>(a, sc.LPL, sc.K, blocks, stream);
      else
        launch_full<SRC_COST, OUT_I32>(a, sc.LPL, sc.K, blocks, stream);
    }
  }
  return launched();
}

mpv_status mpv_disparity(const mpv_params* p, const void* agg, int32_t W, int32_t H,
                         const mpv_band* band, int16_t* disp, int16_t* disp_right,
                         int16_t* disp_raw, hipStream_t stream) {
  mpv_status st = check_params(p, false);
  if (st) return st;
  if (!agg || !disp || W < 1 || H < 1 || W > MPV_MAX_WIDTH) return MPV_ERR_INVALID_ARG;
  if ((st = check_band(band, p->num_disp))) return st;
  const bool banded = band && band->lo;
  RedArgs ra{};
  ra.W = W;
  ra.H = H;
  ra.D = p->num_disp;
  ra.stride = banded ? band->cap : p->num_disp;
  ra.bcap = ra.stride;
  ra.lo = banded ? band->lo : nullptr;
  ra.len = banded ? band->len : nullptr;
  ra.absolute = 0;
  ra.agg = agg;
  ra.lr = p->lr_max_diff;
  ra.disp = disp;
  ra.right = disp_right;
  ra.raw = disp_raw;
  if (p->agg_type == MPV_AGG_U16)
    launch_reduce<IN_U16>(ra, stream);
  else
    launch_reduce<IN_I32>(ra, stream);
  return launched();
}

size_t mpv_match_workspace_bytes(const mpv_params* p, int32_t W, int32_t H, const mpv_band* band) {
  if (check_params(p, true) || W < 1 || H < 1 || check_band(band, p->num_disp)) return 0;
  return level_ws(p, W, H, band).total;
}

mpv_status mpv_match(const mpv_params* p, const mpv_image* left, const mpv_image* right,
                     const mpv_band* band, int16_t* disp, int16_t* disp_right, int16_t* disp_raw,
                     void* workspace, size_t workspace_bytes, hipStream_t stream) {
  mpv_status st = check_params(p, true);
  if (st) return st;
  if (!valid_image(left) || !valid_image(right) || !disp) return MPV_ERR_INVALID_ARG;
  if (left->width != right->width || left->height != right->height) return MPV_ERR_INVALID_ARG;
  if (left->width > MPV_MAX_WIDTH) return MPV_ERR_INVALID_ARG;
  if ((st = check_band(band, p->num_disp))) return st;
  const size_t need = level_ws(p, left->width, left->height, band).total;
  if (!workspace || workspace_bytes < need) return MPV_ERR_WORKSPACE;
  return run_level(p, left->data, left->pitch, right->data, right->pitch, left->width,
                   left->height, band, disp, disp_right, disp_raw, (uint8_t*)workspace, 0, stream);
}

size_t mpv_pyramid_workspace_bytes(const mpv_pyramid_params* p, int32_t W, int32_t H) {
  PyrGeom g;
  if (pyr_geom(p, W, H, g)) return 0;
  return pyr_ws(p, g).total;
}

mpv_status mpv_pyramid(const mpv_pyramid_params* p, const mpv_image* left,
                       const mpv_image* right, const mpv_pyramid_out* out, void* workspace,
                       size_t workspace_bytes, hipStream_t stream) {
  if (!valid_image(left) || !valid_image(right) || !out || !out->disp) return MPV_ERR_INVALID_ARG;
  if (left->width != right->width || left->height != right->height) return MPV_ERR_INVALID_ARG;
  PyrGeom g;
  mpv_status st = pyr_geom(p, left->width, left->height, g);
  if (st) return st;
  const PyrWs w = pyr_ws(p, g);
  if (!workspace || workspace_bytes < w.total) return MPV_ERR_WORKSPACE;
  uint8_t* ws = (uint8_t*)workspace;
  const int L = g.L;
  // image pyramid, finest to coarsest
  const uint8_t* li[MPV_MAX_LEVELS];
  const uint8_t* ri[MPV_MAX_LEVELS];
  int lp[MPV_MAX_LEVELS], rp[MPV_MAX_LEVELS];
  li[L - 1] = left->data;
  ri[L - 1] = right->data;
  lp[L - 1] = left->pitch;
  rp[L - 1] = right->pitch;
  for (int l = L - 2; l >= 0; --l) {
    uint8_t* dl = ws + w.img_off[l];
    uint8_t* dr = dl + (size_t)g.W[l] * g.H[l];
    HookScope hs(MPV_STAGE_DOWNSAMPLE, l, stream);
    dim3 gd = pix_grid(g.W[l], g.H[l]);
    gd.z = 2;
    hipLaunchKernelGGL(k_downsample, gd, dim3(256), 0, stream, li[l + 1], lp[l + 1], dl, g.W[l],
                       g.H[l], ri[l + 1], rp[l + 1], dr);
    li[l] = dl;
    ri[l] = dr;
    lp[l] = rp[l] = g.W[l];
  }
  int16_t* lo = (int16_t*)(ws + w.lo_off);
  for (int l = 0; l < L; ++l) {
    int16_t* raw = out->level_raw[l] ? out->level_raw[l] : (int16_t*)(ws + w.raw_off[l]);
    mpv_params lpar = p->base;
    lpar.num_disp = g.D[l];
    mpv_band b{nullptr, nullptr, g.cap[l]};
    if (l > 0) {
      const int16_t* prev = out->level_raw[l - 1] ? out->level_raw[l - 1]
                                                  : (const int16_t*)(ws + w.raw_off[l - 1]);
      HookScope hs(MPV_STAGE_PROPAGATE, l, stream);
      hipLaunchKernelGGL(k_propagate, pix_grid(g.W[l], g.H[l]), dim3(256), 0, stream, prev,
                         g.W[l - 1], g.H[l - 1], g.W[l], g.H[l], g.D[l], p->band_radius, g.cap[l],
                         lo);
      b.lo = lo;
    }
    const bool last = l == L - 1;
    if (last && out->disp_raw && !out->level_raw[l]) raw = out->disp_raw;
    st = run_level(&lpar, li[l], lp[l], ri[l], rp[l], g.W[l], g.H[l], l > 0 ? &b : nullptr,
                   last ? out->disp : nullptr, last ? out->disp_right : nullptr, raw,
                   ws + w.level_off, l, stream);
    if (st) return st;
    if (last && out->disp_raw && out->level_raw[l] && out->disp_raw != out->level_raw[l])
      if (hipMemcpyAsync(out->disp_raw, out->level_raw[l], (size_t)g.W[l] * g.H[l] * sizeof(int16_t),
                         hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return MPV_ERR_DEVICE;
  }
  return launched();
}

mpv_status mpv_set_timing_events(int32_t stage, int32_t level, hipEvent_t before, hipEvent_t after) {
  if (stage < 0 || stage >= MPV_NUM_STAGES || level < -1 || level >= MPV_MAX_LEVELS)
    return MPV_ERR_INVALID_ARG;
  if ((before == nullptr) != (after == nullptr)) return MPV_ERR_INVALID_ARG;
  g_hook[stage].level = before ? level : -2;
  g_hook[stage].before = before;
  g_hook[stage].after = after;
  return MPV_OK;
}

}  // extern "C"
