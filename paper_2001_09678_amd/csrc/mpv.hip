// C-ABI entry points of the MPV stereo library (declared in include/mpv.h).
//
// Host code only validates, sizes the caller's workspace, picks a kernel variant and
// enqueues on the caller's stream through the launchers of launch.hpp; it never
// allocates device memory and synchronises only in mpv_batch_bind.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <new>
#include <optional>
#include <vector>

#include "../../include/mpv.h"
#include "../../include/mpv_lb.h"
#include "launch.hpp"

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
  if (p->agg_type != MPV_AGG_U16 && p->agg_type != MPV_AGG_I32) return MPV_ERR_INVALID_ARG;
  if (p->merge != MPV_MERGE_SUM && p->merge != MPV_MERGE_LAYERED && p->merge != MPV_MERGE_LAYERED_OCC)
    return MPV_ERR_INVALID_ARG;
  if (p->grad_sigma < 0 || p->grad_sigma > 255) return MPV_ERR_INVALID_ARG;
  if (p->data_term != MPV_DATA_CENSUS && p->data_term != MPV_DATA_SSIM) return MPV_ERR_INVALID_ARG;
  // the fused path scans an SSIM cost volume for the sum of the paths with constant weights
  if (fused && p->data_term == MPV_DATA_SSIM && (p->merge != MPV_MERGE_SUM || p->grad_sigma != 0))
    return MPV_ERR_UNSUPPORTED;
  if (p->merge != MPV_MERGE_SUM) {
    if (p->num_paths < 2) return MPV_ERR_INVALID_ARG;
    // layer k's merged energies are at most 24 + (k+1)*lambda*tau (each pass adds at most
    // lambda*tau to its data term's range; the doubled weight of the occlusion strategy
    // enters one pass of the first layer), and every stored partial must fit a byte
    const long m = std::max(p->num_paths / 2, p->merge == MPV_MERGE_LAYERED_OCC ? 2 : 1);
    if (fused && 24 + m * lt > 255) return MPV_ERR_UNSUPPORTED;
  }
  if (fused ? (24 + lt > 255) : (lt > 4000)) return MPV_ERR_UNSUPPORTED;
  return MPV_OK;
}

mpv_status check_sched(const mpv_schedule& s) {
  const bool wpb = s.waves_per_block == 0 || s.waves_per_block == 1 || s.waves_per_block == 2 ||
                   s.waves_per_block == 4;
  const bool fl = s.full_lanes == 0 || s.full_lanes == 16 || s.full_lanes == 32 || s.full_lanes == 64;
  const bool bl = s.band_lanes == 0 || s.band_lanes == MPV_BAND_LANES_LINE || s.band_lanes == 16 ||
                  s.band_lanes == 32 || s.band_lanes == 64;
  return (wpb && fl && bl && (s.order == 0 || s.order == 1)) ? MPV_OK : MPV_ERR_INVALID_ARG;
}

mpv_status check_band(const mpv_band* b, int D) {
  if (!b || !b->lo) return MPV_OK;
  if (b->cap < 1 || b->cap > D) return MPV_ERR_INVALID_ARG;
  return MPV_OK;
}

mpv_status launched() { return hipGetLastError() == hipSuccess ? MPV_OK : MPV_ERR_DEVICE; }

// ---- timing hook -------------------------------------------------------------------------
struct TimingHook {
  int level = -2;  // -2: unset
  hipEvent_t before = nullptr, after = nullptr;
};
TimingHook g_hook[MPV_NUM_STAGES];

struct HookScope {  // records the stage's events around the launches made in its lifetime
  const TimingHook* h;
  hipStream_t s;
  // level ALL_LEVELS: one launch that serves every level, bracketed whatever level is hooked
  static constexpr int ALL_LEVELS = -2;
  HookScope(int stage, int level, hipStream_t st) : h(nullptr), s(st) {
    const TimingHook& t = g_hook[stage];
    if (t.before && (t.level == -1 || t.level == level || level == ALL_LEVELS)) {
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
FullLayout full_layout(int D, int lanes) {
  if (lanes) {
    const int K = (D + 2 * lanes - 1) / (2 * lanes);
    if (mpvl::full_layout_ok(lanes, K)) return {lanes, K};
  }
  if (D <= 32) return {16, 1};
  if (D <= 64) return {32, 1};
  if (D <= 128) return {64, 1};
  return {64, 2};
}
// Widest padded range any layout may use for D (sizes the census margin).
int max_dpad(int D) { return std::max(2 * 64 * ((D + 127) / 128), 64); }

// Smallest lane group that holds a band of `cap` plus tau-1 neighbours on each side and one
// spare lane (or the requested one if it does); 0 if none. The spare last lane's envelope is
// always absent, and the banded scans read it for every source position outside the group.
int band_lanes(int cap, int te, int want) {
  const int need = cap + 2 * (te - 1);
  if (want && need < want) return want;
  if (need < 16) return 16;
  if (need < 32) return 32;
  if (need < 64) return 64;
  return 0;
}

struct ScanChoice {
  bool banded_kernel;  // k_scan_band
  int LPL, K;
  int capP;  // partial slots per pixel
  bool absolute;
  bool masked;  // full-range kernel with band masks
  // one line per lane for the directions with dy != 0 where the scan source allows it
  // (census, sum of the paths, constant weights); 16-lane groups otherwise
  bool line;
};
// line_ok: the level may run one line per lane (a batched level with the census data term,
// the sum of the paths and constant weights); it then stores 12 partial slots per pixel, or
// six-bit slots in PART6_PITCH bytes where every normalised energy, at most
// 24 + lambda*tau, fits six bits.
ScanChoice choose_scan(int D, const mpv_band* band, int tau, const mpv_schedule& sc, bool line_ok = false,
                       int lambda = 0) {
  const int te = tau_eff(tau, D);
  if (band && band->lo) {
    if (line_ok && sc.band_lanes == MPV_BAND_LANES_LINE && !band->len && mpvl::band_line_ok(band->cap, te)) {
      const bool six = 24 + (long)lambda * te <= 63 && band->cap <= PART6_SLOTS;
      return {true, 16, 1, six ? PART6_PITCH : 12, false, false, true};
    }
    const int lpl = band_lanes(band->cap, te, sc.band_lanes == MPV_BAND_LANES_LINE ? 0 : sc.band_lanes);
    if (lpl) return {true, lpl, 1, lpl, false, false};
    FullLayout f = full_layout(D, sc.full_lanes);
    return {false, f.LPL, f.K, f.dpad(), true, true};
  }
  FullLayout f = full_layout(D, sc.full_lanes);
  return {false, f.LPL, f.K, f.dpad(), false, false};
}

const int kDX[8] = {+1, -1, 0, 0, +1, -1, -1, +1};
const int kDY[8] = {0, 0, +1, -1, +1, -1, +1, -1};
int num_lines_host(int r, int W, int H) { return kDY[r] == 0 ? H : (kDX[r] == 0 ? W : W + H - 1); }
int line_len_host(int r, int W, int H) {
  return kDY[r] == 0 ? W : (kDX[r] == 0 ? H : std::min(W, H));
}

// Fill the direction list and wave prefix of a descriptor; returns its number of waves.
int plan_dirs(ScanArgs& a, const int* dirs, int ndir, int LPL) {
  a.ndir = ndir;
  int waves = 0;
  for (int i = 0; i < ndir; ++i) {
    a.dir[i] = dirs[i];
    a.gprefix[i] = waves;
    waves += (num_lines_host(dirs[i], a.W, a.H) + (64 / LPL) - 1) / (64 / LPL);
  }
  a.gprefix[ndir] = waves;
  for (int i = ndir; i < 8; ++i) a.dir[i] = 0;
  return waves;
}

int wpb_of(const mpv_schedule& s) { return s.waves_per_block ? s.waves_per_block : 1; }

void launch_scan(const ScanArgs& a, const ScanChoice& c, int src, int out, const mpv_schedule& s,
                 hipStream_t st) {
  if (src_grad(src)) {
    if (c.banded_kernel)
      mpvl::scan_band_grad(a, src, c.LPL, a.len != nullptr, wpb_of(s), st);
    else
      mpvl::scan_full_grad(a, src, c.LPL, c.K, c.masked, wpb_of(s), st);
  } else if (src == SRC_MERGE || src == SRC_CENSUS_OCC) {
    if (c.banded_kernel)
      mpvl::scan_band_layered(a, src, c.LPL, a.len != nullptr, wpb_of(s), st);
    else
      mpvl::scan_full_layered(a, src, c.LPL, c.K, c.masked, wpb_of(s), st);
  } else if (c.banded_kernel) {
    mpvl::scan_band(a, c.LPL, src, out, a.len != nullptr, wpb_of(s), st);
  } else {
    mpvl::scan_full(a, c.LPL, c.K, src, out, c.masked, wpb_of(s), st);
  }
}

// ---- one fused level ---------------------------------------------------------------------
struct LevelWs {
  size_t census_off, part_off, total;
  int cpitch, cmargin;
  ScanChoice sc;
  // scans address one census image and one direction's partials with 32-bit offsets, and
  // keep unnormalised energies of lines up to MPV_MAX_HEIGHT long in 32 bits
  bool fits;
};

// own_census: the level workspace holds the census of both views (false when the caller
// computed them elsewhere in the same layout).
LevelWs level_ws(const mpv_params* p, int W, int H, const mpv_band* band, const mpv_schedule& s,
                 bool own_census = true, bool batched = false) {
  LevelWs w{};
  const bool line_ok = batched && p->data_term == MPV_DATA_CENSUS && p->merge == MPV_MERGE_SUM &&
                       p->grad_sigma == 0;
  w.sc = choose_scan(p->num_disp, band, p->tau, s, line_ok, p->lambda);
  // left census margin: covers x - d for every lane of a full-range (padded range) or
  // banded (band start <= D-1, up to 64 lanes) scan
  w.cmargin = (int)align_up((size_t)std::max(max_dpad(p->num_disp), p->num_disp + 64) + 1, 16);
  w.cpitch = w.cmargin + W;
  w.census_off = 0;
  const size_t cen = align_up((size_t)H * w.cpitch * sizeof(uint32_t));
  w.part_off = w.census_off + (own_census ? 2 * cen : 0);
  if (p->data_term == MPV_DATA_SSIM)  // the level's SSIM cost volume [H][W][cap] instead
    w.part_off = align_up((size_t)H * W * ((band && band->lo) ? band->cap : p->num_disp));
  // partial volumes, then a 256 B sink for stores past a line's end
  w.total = w.part_off + align_up((size_t)p->num_paths * H * W * w.sc.capP) + ALIGN;
  w.fits = (size_t)H * W * w.sc.capP <= 0x7FFFFFFFu && cen <= 0x7FFFFFFFu && H <= MPV_MAX_HEIGHT;
  return w;
}

ScanArgs level_scan_args(const mpv_params* p, int W, int H, const mpv_band* band,
                         const LevelWs& lw, uint8_t* ws) {
  ScanArgs a{};
  a.W = W;
  a.H = H;
  a.D = p->num_disp;
  a.cap = (band && band->lo) ? band->cap : p->num_disp;
  a.lambda = p->lambda;
  a.tau = tau_eff(p->tau, p->num_disp);
  if (ws) {
    a.cl = (const uint32_t*)(ws + lw.census_off);
    a.cr = a.cl + align_up((size_t)H * lw.cpitch * sizeof(uint32_t)) / sizeof(uint32_t);
    a.part = ws + lw.part_off;
  }
  a.cpitch = lw.cpitch;
  a.cmargin = lw.cmargin;
  a.lo = band ? band->lo : nullptr;
  a.len = (band && band->lo) ? band->len : nullptr;
  a.capP = lw.sc.capP;
  a.part_stride = (long long)H * W * lw.sc.capP;
  a.dir_base = 0;
  a.npd = p->num_paths;
  a.up_dir = -1;
  return a;
}

// Band of the next finer level, written by this level's reduce.
struct NextBand {
  int16_t* lo;
  int W, H, D, R, cap;
};

RedArgs level_red_args(const mpv_params* p, const ScanArgs& a, const LevelWs& lw, int16_t* disp,
                       int16_t* right, int16_t* raw, const NextBand* nb = nullptr) {
  RedArgs ra{};
  ra.W = a.W;
  ra.H = a.H;
  ra.D = p->num_disp;
  ra.stride = lw.sc.capP;
  ra.bcap = a.cap;
  ra.lo = a.lo;
  ra.len = a.len;
  ra.absolute = lw.sc.absolute ? 1 : 0;
  ra.part = a.part;
  ra.part_stride = a.part_stride;
  ra.npart = p->num_paths;
  ra.lr = p->lr_max_diff;
  ra.need_lr = (disp || right) ? 1 : 0;
  ra.disp = disp;
  ra.right = right;
  ra.raw = raw;
  if (nb) {
    ra.nlo = nb->lo;
    ra.nW = nb->W;
    ra.nH = nb->H;
    ra.nD = nb->D;
    ra.nR = nb->R;
    ra.ncap = nb->cap;
  }
  return ra;
}

// Layer k of a layered merge (Section 3.2 / Table alg) over the scan arguments of a level:
// directions 2k, 2k+1 into partial volumes 2k, 2k+1; the data term is the census cost for
// k = 0 (with the occlusion weight on the left-to-right pass for MPV_MERGE_LAYERED_OCC)
// and the merge of layer k-1's two volumes (min after the horizontal layer, floor mean
// after the others) for k > 0. Returns the scan source.
int layered_layer(const mpv_params* p, ScanArgs& b, int k) {
  b.dir_base = 2 * k;
  if (k == 0) {
    b.up_dir = p->merge == MPV_MERGE_LAYERED_OCC ? 0 : -1;
    return b.up_dir >= 0 ? SRC_CENSUS_OCC : SRC_CENSUS;
  }
  b.msrc = b.part ? b.part + (size_t)(2 * k - 2) * b.part_stride : nullptr;  // null: planning only
  b.mop = k == 1 ? MERGE_MIN : MERGE_MEAN;
  return SRC_MERGE;
}

// The reduce of a layered merge decides on the last layer's merge of its two volumes.
void layered_reduce(const mpv_params* p, RedArgs& ra) {
  const int nl = p->num_paths / 2;
  ra.part = ra.part + (size_t)(2 * nl - 2) * ra.part_stride;
  ra.npart = 2;
  ra.merge = 1 + (nl == 1 ? MERGE_MIN : MERGE_MEAN);
}

// census(L), census(R) -> all P directions -> reduce. disp may be null (intermediate level).
// gimg/gpitch: the left image of the level for gradient-weighted transitions (defaults to L).
mpv_status run_level(const mpv_params* p, const uint8_t* L, int lpitch, const uint8_t* R,
                     int rpitch, int W, int H, const mpv_band* band, int16_t* disp,
                     int16_t* right, int16_t* raw, uint8_t* ws, int level,
                     const mpv_schedule& sched, hipStream_t s, const NextBand* nb = nullptr,
                     uint32_t* const* cen = nullptr, const uint8_t* gimg = nullptr,
                     int gpitch = 0, const CenPyr* fuse = nullptr, int cen0 = 0, int ncen = 0) {
  const LevelWs lw = level_ws(p, W, H, band, sched, cen == nullptr);
  ScanArgs a = level_scan_args(p, W, H, band, lw, ws);
  const int grad = p->grad_sigma > 0 ? SRC_GRAD : 0;
  if (grad) {  // eq. EU: transitions weighted by the left image's gradient along the path
    a.img = gimg ? gimg : L;
    a.ipitch = gimg ? gpitch : lpitch;
    a.sigma = p->grad_sigma;
  }
  const bool ssim = p->data_term == MPV_DATA_SSIM;
  int data = SRC_CENSUS;  // scan source of the data term
  if (ssim) {  // the SSIM cost volume of the level, computed once, read by every direction
    HookScope hs(MPV_STAGE_CENSUS, level, s);
    uint8_t* cv = ws + lw.census_off;
    mpvl::cost_ssim(L, lpitch, R, rpitch, W, H, a.lo, a.len, a.cap, a.D, cv, s);
    a.cost = cv;
    a.cl = a.cr = nullptr;
    data = SRC_COST;
  } else if (cen) {  // census computed beforehand, in the same layout (cpitch, cmargin)
    a.cl = cen[0];
    a.cr = cen[1];
  } else {
    HookScope hs(MPV_STAGE_CENSUS, level, s);
    mpvl::census(L, lpitch, R, rpitch, W, H, (uint32_t*)a.cl, (uint32_t*)a.cr, lw.cpitch,
                 lw.cmargin, s);
  }
  const int nl = p->num_paths / 2;  // layers of a layered merge
  {
    HookScope hs(MPV_STAGE_SCAN, level, s);
    if (p->merge == MPV_MERGE_SUM) {
      int dirs[8];
      for (int i = 0; i < p->num_paths; ++i) dirs[i] = i;
      plan_dirs(a, dirs, p->num_paths, lw.sc.LPL);
      if (fuse && !ssim && !lw.sc.banded_kernel && !lw.sc.masked)  // finer census beside this scan
        mpvl::scan_full_cen(a, SRC_CENSUS | grad, *fuse, cen0, ncen, lw.sc.LPL, lw.sc.K, wpb_of(sched), s);
      else
        launch_scan(a, lw.sc, data | grad, OUT_PART, sched, s);
    } else {
      // Section 3.2 / Table alg: one dependent launch per layer
      for (int k = 0; k < nl; ++k) {
        ScanArgs b = a;
        const int src = layered_layer(p, b, k);
        const int pair[2] = {2 * k, 2 * k + 1};
        plan_dirs(b, pair, 2, lw.sc.LPL);
        if (k == 0 && fuse && !lw.sc.banded_kernel && !lw.sc.masked)  // finer census beside it
          mpvl::scan_full_cen(b, src | grad, *fuse, cen0, ncen, lw.sc.LPL, lw.sc.K, wpb_of(sched), s);
        else
          launch_scan(b, lw.sc, src | grad, OUT_PART, sched, s);
      }
    }
  }
  RedArgs ra = level_red_args(p, a, lw, disp, right, raw, nb);
  if (p->merge != MPV_MERGE_SUM) layered_reduce(p, ra);
  {
    HookScope hs(MPV_STAGE_REDUCE, level, s);
    mpvl::reduce_part(ra, ra.need_lr, s);
  }
  return launched();
}

struct PyrGeom {
  int L;
  int W[MPV_MAX_LEVELS], H[MPV_MAX_LEVELS], D[MPV_MAX_LEVELS], cap[MPV_MAX_LEVELS];
};

mpv_status pyr_geom(const mpv_pyramid_params* p, int D, int W, int H, PyrGeom& g) {
  if (!p) return MPV_ERR_INVALID_ARG;
  mpv_params base = p->base;
  base.num_disp = D;
  mpv_status st = check_params(&base, true);
  if (st) return st;
  if ((st = check_sched(p->sched))) return st;
  if (p->levels < 1 || p->levels > MPV_MAX_LEVELS || p->band_radius < 0) return MPV_ERR_INVALID_ARG;
  if (p->propagation != MPV_PROP_NEAREST && p->propagation != MPV_PROP_PAPER) return MPV_ERR_INVALID_ARG;
  if (p->block < 0 || p->block > MPV_MAX_BLOCK || (p->block & 1)) return MPV_ERR_INVALID_ARG;
  if (W < 1 || H < 1 || W > MPV_MAX_WIDTH) return MPV_ERR_INVALID_ARG;
  g.L = p->levels;
  for (int l = 0; l < g.L; ++l) {
    const int sh = g.L - 1 - l;
    g.W[l] = W >> sh;
    g.H[l] = H >> sh;
    g.D[l] = (D + (1 << sh) - 1) >> sh;
    if (g.W[l] < 1 || g.H[l] < 1) return MPV_ERR_INVALID_ARG;
    g.cap[l] = l == 0 ? g.D[l] : std::min(2 * p->band_radius + 1, g.D[l]);
    mpv_params lp = base;
    lp.num_disp = g.D[l];
    int16_t dummy;
    const mpv_band b{l > 0 ? &dummy : nullptr, nullptr, g.cap[l]};
    if (!level_ws(&lp, g.W[l], g.H[l], l > 0 ? &b : nullptr, p->sched).fits) return MPV_ERR_INVALID_ARG;
  }
  return MPV_OK;
}

struct PyrWs {
  size_t img_off[MPV_MAX_LEVELS];  // left at off, right at off + W*H
  size_t gimg_off[MPV_MAX_LEVELS];  // mpv_pyramid with gradient weights: left image of level l
  size_t raw_off[MPV_MAX_LEVELS];
  size_t lo_off[2];  // band starts: level l reads buffer l & 1, its reduce writes the other
  size_t cen_off[MPV_MAX_LEVELS];  // census of both views of every level (not in unfused mpv_pyramid)
  int cpitch[MPV_MAX_LEVELS], cmargin[MPV_MAX_LEVELS];
  size_t level_off;  // census + partials, reused per level
  size_t total;
};

mpv_params level_params(const mpv_pyramid_params* p, int Dl) {
  mpv_params lp = p->base;
  lp.num_disp = Dl;
  return lp;
}

// MPV_PROP_PAPER: block side of level l (1 .. L-1) of the paper's propagation; 0 = the last
// level's per-pixel interpolation.
int prop_block(const mpv_pyramid_params* p, int L, int l) {
  if (l == L - 1) return 0;
  const int b = p->block ? p->block : 8;
  return std::max(b >> (l - 1), 2);
}

// fused_census (mpv_pyramid): the census of every level is computed up front from the input
// (no coarse images are kept); otherwise coarse images. mpv_pyramid and batches keep every
// level's census apart from the level workspace (batches compute a finer level's census while
// the coarser levels are matched).
PyrWs pyr_ws(const mpv_pyramid_params* p, const PyrGeom& g, bool fused_census = false, bool batched = false) {
  PyrWs w{};
  size_t off = 0;
  const bool cen_levels = fused_census || batched;
  for (int l = 0; l + 1 < g.L && !fused_census; ++l) {
    w.img_off[l] = off;
    off += align_up((size_t)2 * g.W[l] * g.H[l]);
  }
  for (int l = 0; l + 1 < g.L && fused_census && p->base.grad_sigma > 0; ++l) {
    w.gimg_off[l] = off;
    off += align_up((size_t)g.W[l] * g.H[l]);
  }
  for (int l = 0; l < g.L; ++l) {
    w.raw_off[l] = off;
    off += align_up((size_t)g.W[l] * g.H[l] * sizeof(int16_t));
  }
  for (int k = 0; k < 2; ++k) {
    w.lo_off[k] = off;
    off += align_up((size_t)g.W[g.L - 1] * g.H[g.L - 1] * sizeof(int16_t));
  }
  size_t lvl = 0;
  for (int l = 0; l < g.L; ++l) {
    const mpv_params lp = level_params(p, g.D[l]);
    mpv_band b{nullptr, nullptr, g.cap[l]};
    int16_t dummy;
    if (l > 0) b.lo = &dummy;  // only presence matters for sizing
    const LevelWs lw = level_ws(&lp, g.W[l], g.H[l], l > 0 ? &b : nullptr, p->sched, !cen_levels, batched);
    lvl = std::max(lvl, lw.total);
    if (cen_levels) {
      w.cen_off[l] = off;
      w.cpitch[l] = lw.cpitch;
      w.cmargin[l] = lw.cmargin;
      off += 2 * align_up((size_t)g.H[l] * lw.cpitch * sizeof(uint32_t));
    }
  }
  w.level_off = off;
  w.total = off + lvl;
  return w;
}

}  // namespace

// =========================================================================================
// Batch planner
// =========================================================================================
struct mpv_batch_s {
  mpv_pyramid_params p;
  struct Pair {
    mpv_batch_item item;
    PyrGeom g;
    PyrWs w;
    size_t off;  // workspace region of this pair (after the tables)
  };
  std::vector<Pair> pairs;
  size_t table_bytes = 0;  // descriptor tables at the start of the workspace
  // a second table area right after the first holds the tables of mpv_batch_run_items;
  // the pairs' regions start after both
  size_t region_base() const { return 2 * table_bytes; }
  size_t total = 0;
  // mpv_batch_run_items: pinned staging of its tables (a ring, each entry reusable once the
  // event recorded after its upload has completed)
  static constexpr int kStage = 4;
  uint8_t* stage = nullptr;
  hipEvent_t stage_ev[kStage] = {};
  int stage_next = 0;
  uint8_t* ws = nullptr;
  enum Kind { DOWN, CENSUS, SCAN_FULL, SCAN_BAND, REDUCE };
  struct Launch {
    Kind kind;
    int level;
    size_t desc_off, first_off;  // in the table area
    int nseg, units;             // units: waves (scans), blocks (others)
    int LPL, K, tau, stride;
    bool masked;
    int src;  // scans: SRC_CENSUS, or a layered merge's SRC_CENSUS_OCC / SRC_MERGE
    bool line;  // banded scans with one line per lane (bands of cap disparities)
    int cap;
    bool beside;  // runs on the auxiliary stream beside the previous launch: forked from before
                  // it (which is dispatched first), joined after both
    bool early;   // a finer level's census: runs on the census stream from here on, joined
                  // before its level's first scan
  };
  std::vector<Launch> launches;  // execution order
  std::vector<Launch> sub_launches;  // launches of the last mpv_batch_run_items
  // a level's lane-group scan runs beside its one-line-per-lane scan: the two kernels have
  // different register budgets and fill the machine together
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // the finer levels' census runs on a stream of its own while the coarser levels are matched
  hipStream_t caux = nullptr;
  hipEvent_t cfork_ev = nullptr, cjoin_ev[MPV_MAX_LEVELS] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// Descriptor tables and segment prefixes appended to a host image of the table area.
struct TableBuilder {
  std::vector<uint8_t> bytes;
  template <typename T>
  size_t put(const std::vector<T>& v) {
    const size_t off = align_up(bytes.size(), 16);
    bytes.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
};

// Plan every launch of a batch. With ws == nullptr the pointers are left null and only the
// table size matters.
void plan_batch(mpv_batch_s& b, uint8_t* ws, TableBuilder& tb) {
  b.launches.clear();
  const int L = b.p.levels;
  const mpv_schedule& sc = b.p.sched;
  const int n = (int)b.pairs.size();
  auto region = [&](const mpv_batch_s::Pair& pr) -> uint8_t* {
    return ws ? ws + b.region_base() + pr.off : nullptr;
  };
  auto add_pix = [&](mpv_batch_s::Kind kind, int level, std::vector<PixArgs>& d, int views) {
    std::vector<int> first;
    int blocks = 0;
    const int rows = kind == mpv_batch_s::CENSUS ? mpvk::CENSUS_TILE_ROWS : 4;  // tile: 64 x rows pixels
    for (auto& a : d) {
      a.tiles_x = (a.W + 63) / 64;
      a.tiles = a.tiles_x * ((a.H + rows - 1) / rows);
      first.push_back(blocks);
      blocks += a.tiles * views;
    }
    first.push_back(blocks);
    mpv_batch_s::Launch ln{};
    ln.kind = kind;
    ln.level = level;
    ln.desc_off = tb.put(d);
    ln.first_off = tb.put(first);
    ln.nseg = (int)d.size();
    ln.units = blocks;
    b.launches.push_back(ln);
  };
  auto img_at = [&](const mpv_batch_s::Pair& pr, int l, int v, int& pitch) -> const uint8_t* {
    if (l == L - 1) {
      const mpv_image& im = v ? pr.item.right : pr.item.left;
      pitch = im.pitch;
      return im.data;
    }
    pitch = pr.g.W[l];
    uint8_t* r = region(pr);
    return r ? r + pr.w.img_off[l] + (size_t)v * pr.g.W[l] * pr.g.H[l] : nullptr;
  };
  // image pyramids, finest to coarsest
  for (int l = L - 2; l >= 0; --l) {
    std::vector<PixArgs> d;
    for (auto& pr : b.pairs) {
      PixArgs a{};
      a.W = pr.g.W[l];
      a.H = pr.g.H[l];
      for (int v = 0; v < 2; ++v) {
        a.in[v] = img_at(pr, l + 1, v, a.in_pitch[v]);
        int dummy;
        a.out[v] = (void*)img_at(pr, l, v, dummy);
      }
      d.push_back(a);
    }
    add_pix(mpv_batch_s::DOWN, l, d, 2);
  }
  for (int l = 0; l < L; ++l) {
    const bool last = l == L - 1;
    std::vector<PixArgs> cd;
    std::vector<ScanArgs> sargs(n);
    std::vector<LevelWs> lws(n);
    for (int i = 0; i < n; ++i) {
      auto& pr = b.pairs[i];
      uint8_t* r = region(pr);
      const mpv_params lp = level_params(&b.p, pr.g.D[l]);
      static int16_t dummy_lo;
      mpv_band band{l > 0 ? (r ? (const int16_t*)(r + pr.w.lo_off[l & 1]) : &dummy_lo) : nullptr,
                    nullptr, pr.g.cap[l]};
      lws[i] = level_ws(&lp, pr.g.W[l], pr.g.H[l], l > 0 ? &band : nullptr, sc, false, true);
      sargs[i] = level_scan_args(&lp, pr.g.W[l], pr.g.H[l], l > 0 ? &band : nullptr, lws[i],
                                 r ? r + pr.w.level_off : nullptr);
      if (r) {  // the level's census, in its own region
        sargs[i].cl = (const uint32_t*)(r + pr.w.cen_off[l]);
        sargs[i].cr = sargs[i].cl + align_up((size_t)pr.g.H[l] * lws[i].cpitch * sizeof(uint32_t)) / sizeof(uint32_t);
      } else {
        sargs[i].lo = nullptr;
      }
      if (b.p.base.grad_sigma > 0) {  // eq. EU weights from the level's left image
        sargs[i].img = img_at(pr, l, 0, sargs[i].ipitch);
        sargs[i].sigma = b.p.base.grad_sigma;
      }
      PixArgs a{};
      a.W = pr.g.W[l];
      a.H = pr.g.H[l];
      for (int v = 0; v < 2; ++v) a.in[v] = img_at(pr, l, v, a.in_pitch[v]);
      a.out[0] = (void*)sargs[i].cl;
      a.out[1] = (void*)sargs[i].cr;
      a.opitch = lws[i].cpitch;
      a.omargin = lws[i].cmargin;
      cd.push_back(a);
    }
    add_pix(mpv_batch_s::CENSUS, l, cd, 2);
    // scans: pairs grouped by kernel variant, one descriptor per (pair, direction)
    struct Key {
      bool band;
      int LPL, K, tau;
      bool masked;
      int line_cap;  // > 0: one line per lane for the directions with dy != 0, bands of this cap
      int pitch;     // partial slots per pixel (PART6_PITCH: six-bit slots)
      bool operator==(const Key& o) const {
        return band == o.band && LPL == o.LPL && K == o.K && tau == o.tau && masked == o.masked &&
               line_cap == o.line_cap && pitch == o.pitch;
      }
    };
    const bool layered = b.p.base.merge != MPV_MERGE_SUM;
    const int grad = b.p.base.grad_sigma > 0 ? SRC_GRAD : 0;
    auto key_of = [&](int i) {
      const ScanChoice& c = lws[i].sc;
      const bool line = c.line && !layered && !grad;
      return Key{c.banded_kernel, c.LPL, c.K, sargs[i].tau, c.masked, line ? sargs[i].cap : 0, c.capP};
    };
    std::vector<Key> keys;
    for (int i = 0; i < n; ++i)
      if (std::find(keys.begin(), keys.end(), key_of(i)) == keys.end()) keys.push_back(key_of(i));
    // sum: one launch per variant with every direction of every pair; layered merge: the
    // layers in turn, each one launch per variant with its two directions of every pair
    const int nstage = layered ? b.p.base.num_paths / 2 : 1;
    for (int stage = 0; stage < nstage; ++stage)
    for (const Key& k : keys) {
      struct Item {
        ScanArgs a;
        int len;
      };
      std::vector<Item> items;
      int src = SRC_CENSUS;
      for (int i = 0; i < n; ++i) {
        if (!(key_of(i) == k)) continue;
        const int r0 = layered ? 2 * stage : 0, r1 = layered ? 2 * stage + 2 : b.p.base.num_paths;
        for (int r = r0; r < r1; ++r) {
          ScanArgs a = sargs[i];
          if (layered) src = layered_layer(&b.p.base, a, stage);
          a.dir_base = r;
          if (k.line_cap && kDY[r] != 0) {
            plan_dirs(a, &r, 1, 1);
            a.line_lanes = 1;
          } else {
            plan_dirs(a, &r, 1, k.LPL);
          }
          items.push_back({a, line_len_host(r, a.W, a.H)});
        }
      }
      if (sc.order == 1)  // longest lines first: the last waves to start are the short ones
        std::stable_sort(items.begin(), items.end(),
                         [](const Item& x, const Item& y) { return x.len > y.len; });
      // one launch per layout: lane groups, then (line_cap) the one-line-per-lane descriptors
      for (int lines = 0; lines < (k.line_cap ? 2 : 1); ++lines) {
        std::vector<ScanArgs> d;
        std::vector<int> first;
        int waves = 0;
        for (auto& it : items) {
          if (it.a.line_lanes != lines) continue;
          d.push_back(it.a);
          first.push_back(waves);
          waves += it.a.gprefix[1];
        }
        if (d.empty()) continue;
        first.push_back(waves);
        mpv_batch_s::Launch ln{};
        ln.kind = k.band ? mpv_batch_s::SCAN_BAND : mpv_batch_s::SCAN_FULL;
        ln.level = l;
        ln.desc_off = tb.put(d);
        ln.first_off = tb.put(first);
        ln.nseg = (int)d.size();
        ln.units = waves;
        ln.LPL = k.LPL;
        ln.K = k.K;
        ln.tau = k.tau;
        ln.masked = k.masked;
        ln.src = src | grad;
        ln.line = lines == 1;
        ln.cap = k.line_cap;
        ln.stride = k.pitch;
        b.launches.push_back(ln);
      }
      // both layouts present: the line launch first (its long chains start at once), the
      // lane-group launch beside it
      const size_t nl = b.launches.size();
      if (k.line_cap && nl >= 2 && b.launches[nl - 1].line && !b.launches[nl - 2].line &&
          b.launches[nl - 2].kind == mpv_batch_s::SCAN_BAND && b.launches[nl - 2].level == l) {
        std::swap(b.launches[nl - 2], b.launches[nl - 1]);
        b.launches[nl - 1].beside = true;
      }
    }
    // reduce: pairs grouped by partial stride
    std::vector<int> strides;
    for (int i = 0; i < n; ++i)
      if (std::find(strides.begin(), strides.end(), lws[i].sc.capP) == strides.end())
        strides.push_back(lws[i].sc.capP);
    for (int st : strides) {
      std::vector<RedArgs> d;
      std::vector<int> first;
      int rows = 0;
      for (int i = 0; i < n; ++i) {
        if (lws[i].sc.capP != st) continue;
        auto& pr = b.pairs[i];
        uint8_t* r = region(pr);
        const mpv_params lp = level_params(&b.p, pr.g.D[l]);
        int16_t* raw = r ? (int16_t*)(r + pr.w.raw_off[l]) : nullptr;
        NextBand nb{r ? (int16_t*)(r + pr.w.lo_off[(l + 1) & 1]) : nullptr, 0, 0, 0, 0, 0};
        if (!last) {
          nb.W = pr.g.W[l + 1];
          nb.H = pr.g.H[l + 1];
          nb.D = pr.g.D[l + 1];
          nb.R = b.p.band_radius;
          nb.cap = pr.g.cap[l + 1];
        }
        RedArgs ra = level_red_args(&lp, sargs[i], lws[i], last ? pr.item.disp : nullptr,
                                    last ? pr.item.disp_right : nullptr, raw,
                                    last || !r ? nullptr : &nb);
        if (last && pr.item.disp_raw) ra.raw = pr.item.disp_raw;
        if (b.p.base.merge != MPV_MERGE_SUM) layered_reduce(&b.p.base, ra);
        d.push_back(ra);
        first.push_back(rows);
        rows += ra.H;
      }
      first.push_back(rows);
      mpv_batch_s::Launch ln{};
      ln.kind = mpv_batch_s::REDUCE;
      ln.level = l;
      ln.desc_off = tb.put(d);
      ln.first_off = tb.put(first);
      ln.nseg = (int)d.size();
      ln.units = rows;
      ln.stride = st;
      b.launches.push_back(ln);
    }
  }
  // the finer levels' census (each in its own region) starts after the top level's census,
  // beside the coarser levels' scans and reduces
  std::vector<mpv_batch_s::Launch> early, order;
  for (auto& ln : b.launches) {
    if (ln.kind == mpv_batch_s::CENSUS && ln.level > 0) {
      ln.early = true;
      early.push_back(ln);
    } else {
      order.push_back(ln);
    }
  }
  auto top = std::find_if(order.begin(), order.end(), [](const mpv_batch_s::Launch& x) {
    return x.kind == mpv_batch_s::CENSUS && x.level == 0;
  });
  order.insert(top == order.end() ? order.end() : top + 1, early.begin(), early.end());
  b.launches = std::move(order);
}

// mpv_pyramid over the SSIM data term: the coarser images of both views are built first
// (Section 3.4 pyramid, finest to coarsest), then every level computes its SSIM cost volume
// and runs the scans and the reduce on it; the bands propagate as with the census.
mpv_status pyramid_ssim(const mpv_pyramid_params* p, const PyrGeom& g, const PyrWs& w,
                        const mpv_image* left, const mpv_image* right, const mpv_pyramid_out* out,
                        uint8_t* ws, hipStream_t stream) {
  const int L = g.L;
  const uint8_t* img[MPV_MAX_LEVELS][2];
  int pitch[MPV_MAX_LEVELS];
  img[L - 1][0] = left->data;
  img[L - 1][1] = right->data;
  pitch[L - 1] = left->pitch;
  for (int l = L - 2; l >= 0; --l) {
    uint8_t* dl = ws + w.img_off[l];
    uint8_t* dr = dl + (size_t)g.W[l] * g.H[l];
    HookScope hs(MPV_STAGE_DOWNSAMPLE, l, stream);
    if (l == L - 2 && left->pitch != right->pitch) {  // two launches: the views' pitches differ
      mpvl::downsample(left->data, left->pitch, dl, nullptr, 0, nullptr, g.W[l], g.H[l], stream);
      mpvl::downsample(right->data, right->pitch, dr, nullptr, 0, nullptr, g.W[l], g.H[l], stream);
    } else {
      mpvl::downsample(img[l + 1][0], pitch[l + 1], dl, img[l + 1][1], pitch[l + 1], dr, g.W[l], g.H[l],
                       stream);
    }
    img[l][0] = dl;
    img[l][1] = dr;
    pitch[l] = g.W[l];
  }
  for (int l = 0; l < L; ++l) {
    int16_t* raw = out->level_raw[l] ? out->level_raw[l] : (int16_t*)(ws + w.raw_off[l]);
    const mpv_params lpar = level_params(p, g.D[l]);
    mpv_band b{l > 0 ? (const int16_t*)(ws + w.lo_off[l & 1]) : nullptr, nullptr, g.cap[l]};
    const bool last = l == L - 1;
    NextBand nb{(int16_t*)(ws + w.lo_off[(l + 1) & 1]), 0, 0, 0, 0, 0};
    if (!last) {
      nb.W = g.W[l + 1];
      nb.H = g.H[l + 1];
      nb.D = g.D[l + 1];
      nb.R = p->band_radius;
      nb.cap = g.cap[l + 1];
    }
    if (last && out->disp_raw && !out->level_raw[l]) raw = out->disp_raw;
    const bool paper = p->propagation == MPV_PROP_PAPER;
    const mpv_status st = run_level(&lpar, img[l][0], pitch[l], img[l][1], last ? right->pitch : pitch[l],
                                    g.W[l], g.H[l], l > 0 ? &b : nullptr, last ? out->disp : nullptr,
                                    last ? out->disp_right : nullptr, raw, ws + w.level_off, l, p->sched,
                                    stream, (last || paper) ? nullptr : &nb);
    if (st) return st;
    if (paper && !last) {
      HookScope hs(MPV_STAGE_PROPAGATE, l, stream);
      const PropArgs pa{raw, g.W[l], g.H[l], nb.lo, nb.W, nb.H, nb.D, nb.R, nb.cap, prop_block(p, L, l + 1)};
      mpvl::propagate(pa, stream);
    }
    if (last && out->disp_raw && out->level_raw[l] && out->disp_raw != out->level_raw[l])
      if (hipMemcpyAsync(out->disp_raw, out->level_raw[l], (size_t)g.W[l] * g.H[l] * sizeof(int16_t),
                         hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return MPV_ERR_DEVICE;
  }
  return launched();
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
  mpvl::census(img->data, img->pitch, nullptr, 0, img->width, img->height, census, nullptr,
               img->width, 0, stream);
  return launched();
}

mpv_status mpv_downsample(const mpv_image* img, uint8_t* out, hipStream_t stream) {
  if (!valid_image(img) || !out) return MPV_ERR_INVALID_ARG;
  const int w = img->width / 2, h = img->height / 2;
  if (w < 1 || h < 1) return MPV_ERR_INVALID_ARG;
  mpvl::downsample(img->data, img->pitch, out, nullptr, 0, nullptr, w, h, stream);
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
  (p->data_term == MPV_DATA_SSIM ? mpvl::cost_ssim : mpvl::cost)(
      left->data, left->pitch, right->data, right->pitch, W, H, banded ? band->lo : nullptr,
      banded ? band->len : nullptr, banded ? band->cap : p->num_disp, p->num_disp, cost, stream);
  return launched();
}

mpv_status mpv_aggregate(const mpv_params* p, const uint8_t* cost, int32_t W, int32_t H,
                         const mpv_band* band, uint32_t path_mask, void* agg,
                         hipStream_t stream) {
  mpv_status st = check_params(p, false);
  if (st) return st;
  if (p->merge != MPV_MERGE_SUM || p->grad_sigma != 0) return MPV_ERR_UNSUPPORTED;
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
  if (p->agg_type == MPV_AGG_U16)
    mpvl::fill_u16((uint16_t*)agg, n, 0xFFFF, stream);
  else
    mpvl::fill_i32((int32_t*)agg, n, 0x7FFFFFFF, stream);
  const mpv_schedule dflt{};
  const ScanChoice sc = choose_scan(p->num_disp, band, p->tau, dflt);
  const int out = p->agg_type == MPV_AGG_U16 ? OUT_U16 : OUT_I32;
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
    a.npd = 1;
    plan_dirs(a, &dirs[i], 1, sc.LPL);
    launch_scan(a, sc, SRC_COST, out, dflt, stream);
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
  ra.need_lr = 1;
  ra.disp = disp;
  ra.right = disp_right;
  ra.raw = disp_raw;
  mpvl::reduce_agg(ra, p->agg_type == MPV_AGG_U16 ? IN_U16 : IN_I32, stream);
  return launched();
}

size_t mpv_match_workspace_bytes(const mpv_params* p, int32_t W, int32_t H, const mpv_band* band) {
  if (check_params(p, true) || W < 1 || H < 1 || W > MPV_MAX_WIDTH || check_band(band, p->num_disp))
    return 0;
  const LevelWs lw = level_ws(p, W, H, band, mpv_schedule{});
  return lw.fits ? lw.total : 0;
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
  const mpv_schedule dflt{};
  const LevelWs lw = level_ws(p, left->width, left->height, band, dflt);
  if (!lw.fits) return MPV_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < lw.total) return MPV_ERR_WORKSPACE;
  return run_level(p, left->data, left->pitch, right->data, right->pitch, left->width,
                   left->height, band, disp, disp_right, disp_raw, (uint8_t*)workspace, 0, dflt,
                   stream);
}

size_t mpv_pyramid_workspace_bytes(const mpv_pyramid_params* p, int32_t W, int32_t H) {
  PyrGeom g;
  if (!p || pyr_geom(p, p->base.num_disp, W, H, g)) return 0;
  return pyr_ws(p, g, p->base.data_term != MPV_DATA_SSIM).total;
}

mpv_status mpv_pyramid(const mpv_pyramid_params* p, const mpv_image* left,
                       const mpv_image* right, const mpv_pyramid_out* out, void* workspace,
                       size_t workspace_bytes, hipStream_t stream) {
  if (!valid_image(left) || !valid_image(right) || !out || !out->disp || !p)
    return MPV_ERR_INVALID_ARG;
  if (left->width != right->width || left->height != right->height) return MPV_ERR_INVALID_ARG;
  PyrGeom g;
  mpv_status st = pyr_geom(p, p->base.num_disp, left->width, left->height, g);
  if (st) return st;
  const bool ssim = p->base.data_term == MPV_DATA_SSIM;
  const PyrWs w = pyr_ws(p, g, !ssim);
  if (!workspace || workspace_bytes < w.total) return MPV_ERR_WORKSPACE;
  uint8_t* ws = (uint8_t*)workspace;
  const int L = g.L;
  if (ssim) return pyramid_ssim(p, g, w, left, right, out, ws, stream);
  // census of every level of both views, built from the input in one launch
  CenPyr cp{};
  cp.img[0] = left->data;
  cp.img[1] = right->data;
  cp.pitch[0] = left->pitch;
  cp.pitch[1] = right->pitch;
  cp.L = L;
  uint32_t* cen[MPV_MAX_LEVELS][2];
  int blocks = 0;
  for (int l = 0; l < L; ++l) {
    cp.W[l] = g.W[l];
    cp.H[l] = g.H[l];
    const size_t view = align_up((size_t)g.H[l] * w.cpitch[l] * sizeof(uint32_t));
    cen[l][0] = (uint32_t*)(ws + w.cen_off[l]);
    cen[l][1] = (uint32_t*)(ws + w.cen_off[l] + view);
    cp.out[l][0] = cen[l][0];
    cp.out[l][1] = cen[l][1];
    cp.opitch[l] = w.cpitch[l];
    cp.omargin[l] = w.cmargin[l];
    cp.tiles_x[l] = (g.W[l] + 63) / 64;
    cp.first[l] = blocks;
    blocks += cp.tiles_x[l] * ((g.H[l] + 3) / 4);
    // gradient-weighted transitions need the coarse levels' left images (the finest is the input)
    cp.limg[l] = (p->base.grad_sigma > 0 && l + 1 < L) ? ws + w.gimg_off[l] : nullptr;
  }
  cp.first[L] = blocks;
  // The top level's (first) scan launch also builds the finer levels' census (its few waves
  // leave the chip idle), so only the top level's census runs first.
  const bool fuse = L > 1;
  {
    HookScope hs(MPV_STAGE_CENSUS, HookScope::ALL_LEVELS, stream);
    mpvl::census_pyr(cp, stream, fuse ? cp.first[1] : -1);
  }
  for (int l = 0; l < L; ++l) {
    int16_t* raw = out->level_raw[l] ? out->level_raw[l] : (int16_t*)(ws + w.raw_off[l]);
    const mpv_params lpar = level_params(p, g.D[l]);
    // this level's band was written by the coarser level's reduce (Section 3.4 propagation)
    mpv_band b{l > 0 ? (const int16_t*)(ws + w.lo_off[l & 1]) : nullptr, nullptr, g.cap[l]};
    const bool last = l == L - 1;
    NextBand nb{(int16_t*)(ws + w.lo_off[(l + 1) & 1]), 0, 0, 0, 0, 0};
    if (!last) {
      nb.W = g.W[l + 1];
      nb.H = g.H[l + 1];
      nb.D = g.D[l + 1];
      nb.R = p->band_radius;
      nb.cap = g.cap[l + 1];
    }
    if (last && out->disp_raw && !out->level_raw[l]) raw = out->disp_raw;
    // nearest propagation rides in this level's reduce; the paper's runs after it
    const bool paper = p->propagation == MPV_PROP_PAPER;
    st = run_level(&lpar, nullptr, 0, nullptr, 0, g.W[l], g.H[l], l > 0 ? &b : nullptr,
                   last ? out->disp : nullptr, last ? out->disp_right : nullptr, raw,
                   ws + w.level_off, l, p->sched, stream, (last || paper) ? nullptr : &nb, cen[l],
                   last ? left->data : cp.limg[l], last ? left->pitch : g.W[l],
                   fuse && l == 0 ? &cp : nullptr, cp.first[1], cp.first[L] - cp.first[1]);
    if (st) return st;
    if (paper && !last) {
      HookScope hs(MPV_STAGE_PROPAGATE, l, stream);
      const PropArgs pa{raw, g.W[l], g.H[l], nb.lo, nb.W, nb.H, nb.D, nb.R, nb.cap, prop_block(p, L, l + 1)};
      mpvl::propagate(pa, stream);
    }
    if (last && out->disp_raw && out->level_raw[l] && out->disp_raw != out->level_raw[l])
      if (hipMemcpyAsync(out->disp_raw, out->level_raw[l], (size_t)g.W[l] * g.H[l] * sizeof(int16_t),
                         hipMemcpyDeviceToDevice, stream) != hipSuccess)
        return MPV_ERR_DEVICE;
  }
  return launched();
}

// ---- batch -------------------------------------------------------------------------------
mpv_status mpv_batch_create(const mpv_pyramid_params* p, const mpv_batch_item* items, int32_t n,
                            mpv_batch* out) {
  if (!p || !items || n < 1 || !out) return MPV_ERR_INVALID_ARG;
  if (p->propagation == MPV_PROP_PAPER || p->base.data_term != MPV_DATA_CENSUS) return MPV_ERR_UNSUPPORTED;
  mpv_batch_s* b = new (std::nothrow) mpv_batch_s();
  if (!b) return MPV_ERR_INVALID_ARG;
  b->p = *p;
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    const mpv_batch_item& it = items[i];
    if (!valid_image(&it.left) || !valid_image(&it.right) || !it.disp ||
        it.left.width != it.right.width || it.left.height != it.right.height) {
      delete b;
      return MPV_ERR_INVALID_ARG;
    }
    mpv_batch_s::Pair pr{};
    pr.item = it;
    const mpv_status st = pyr_geom(p, it.num_disp, it.left.width, it.left.height, pr.g);
    if (st) {
      delete b;
      return st;
    }
    pr.w = pyr_ws(p, pr.g, false, true);
    pr.off = off;
    off += align_up(pr.w.total);
    b->pairs.push_back(pr);
  }
  TableBuilder tb;
  plan_batch(*b, nullptr, tb);
  b->table_bytes = align_up(tb.bytes.size());
  b->total = b->region_base() + off;
  *out = b;
  return MPV_OK;
}

size_t mpv_batch_workspace_bytes(mpv_batch b) { return b ? b->total : 0; }

mpv_status mpv_batch_bind(mpv_batch b, void* workspace, size_t bytes, hipStream_t stream) {
  if (!b || !workspace) return MPV_ERR_INVALID_ARG;
  if (bytes < b->total) return MPV_ERR_WORKSPACE;
  b->ws = (uint8_t*)workspace;
  TableBuilder tb;
  plan_batch(*b, b->ws, tb);
  if (align_up(tb.bytes.size()) > b->table_bytes) return MPV_ERR_WORKSPACE;
  const bool side = std::any_of(b->launches.begin(), b->launches.end(),
                                [](const mpv_batch_s::Launch& x) { return x.beside; });
  if (side && !b->aux) {  // without them the launches run one after the other on the stream
    if (hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join_ev, hipEventDisableTiming) != hipSuccess)
      return MPV_ERR_DEVICE;
  }
  const bool early = std::any_of(b->launches.begin(), b->launches.end(),
                                 [](const mpv_batch_s::Launch& x) { return x.early; });
  if (early && !b->caux) {
    if (hipStreamCreateWithFlags(&b->caux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->cfork_ev, hipEventDisableTiming) != hipSuccess)
      return MPV_ERR_DEVICE;
    for (int l = 0; l < MPV_MAX_LEVELS; ++l)
      if (hipEventCreateWithFlags(&b->cjoin_ev[l], hipEventDisableTiming) != hipSuccess) return MPV_ERR_DEVICE;
  }
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    (void)hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  if (hipMemcpyAsync(b->ws, tb.bytes.data(), tb.bytes.size(), hipMemcpyHostToDevice, stream) !=
      hipSuccess)
    return MPV_ERR_DEVICE;
  return hipStreamSynchronize(stream) == hipSuccess ? MPV_OK : MPV_ERR_DEVICE;
}

}  // extern "C"

namespace {
// Enqueue planned launches whose tables start at `tables` in device memory.
mpv_status run_launches(mpv_batch b, const std::vector<mpv_batch_s::Launch>& launches, const uint8_t* tables,
                        hipStream_t s) {
  const int wpb = wpb_of(b->p.sched);
  // the consecutive launches of one stage at one level (kernel variants, layers of a
  // layered merge) are bracketed together by the timing hook
  std::optional<HookScope> hs;
  int hs_stage = -1, hs_level = -1;
  bool cpend[MPV_MAX_LEVELS] = {};  // the level's census runs on the census stream
  for (size_t li = 0; li < launches.size(); ++li) {
    const auto& ln = launches[li];
    const void* desc = tables + ln.desc_off;
    const int* first = (const int*)(tables + ln.first_off);
    const int stage = ln.kind == mpv_batch_s::DOWN     ? MPV_STAGE_DOWNSAMPLE
                      : ln.kind == mpv_batch_s::CENSUS ? MPV_STAGE_CENSUS
                      : ln.kind == mpv_batch_s::REDUCE ? MPV_STAGE_REDUCE
                                                       : MPV_STAGE_SCAN;
    const bool scan = ln.kind == mpv_batch_s::SCAN_FULL || ln.kind == mpv_batch_s::SCAN_BAND;
    if (scan && cpend[ln.level]) {  // join the level's census (before the stage's timing event)
      if (hipStreamWaitEvent(s, b->cjoin_ev[ln.level], 0) != hipSuccess) return MPV_ERR_DEVICE;
      cpend[ln.level] = false;
    }
    hipStream_t s_main = s;
    const bool on_caux = ln.early && b->caux;
    if (on_caux) {  // fork: the census stream starts after everything before
      if (hipEventRecord(b->cfork_ev, s) != hipSuccess || hipStreamWaitEvent(b->caux, b->cfork_ev, 0) != hipSuccess)
        return MPV_ERR_DEVICE;
      s = b->caux;
    }
    if (stage != hs_stage || ln.level != hs_level) {
      hs.reset();
      hs.emplace(stage, ln.level, s);
      hs_stage = stage;
      hs_level = ln.level;
    }
    const bool fork = b->aux && li + 1 < launches.size() && launches[li + 1].beside;
    if (fork && hipEventRecord(b->fork_ev, s) != hipSuccess) return MPV_ERR_DEVICE;  // before this one
    if (ln.beside && b->aux) {  // the auxiliary stream starts where the previous launch did
      if (hipStreamWaitEvent(b->aux, b->fork_ev, 0) != hipSuccess) return MPV_ERR_DEVICE;
      s = b->aux;
    }
    switch (ln.kind) {
      case mpv_batch_s::DOWN: {
        mpvl::downsample_batch({(const PixArgs*)desc, first, ln.nseg}, ln.units, s);
        break;
      }
      case mpv_batch_s::CENSUS: {
        mpvl::census_batch({(const PixArgs*)desc, first, ln.nseg}, ln.units, s);
        break;
      }
      case mpv_batch_s::SCAN_FULL: {
        if (src_grad(ln.src))
          mpvl::scan_full_batch_grad({(const ScanArgs*)desc, first, ln.nseg}, ln.src, ln.units, ln.LPL,
                                     ln.K, ln.tau, ln.masked, wpb, s);
        else if (ln.src == SRC_CENSUS)
          mpvl::scan_full_batch({(const ScanArgs*)desc, first, ln.nseg}, ln.units, ln.LPL, ln.K,
                                ln.tau, ln.masked, wpb, s);
        else
          mpvl::scan_full_batch_layered({(const ScanArgs*)desc, first, ln.nseg}, ln.src, ln.units,
                                        ln.LPL, ln.K, ln.tau, ln.masked, wpb, s);
        break;
      }
      case mpv_batch_s::SCAN_BAND: {
        if (ln.line)
          mpvl::scan_lane_batch({(const ScanArgs*)desc, first, ln.nseg}, ln.units, ln.cap, ln.tau,
                                ln.stride == PART6_PITCH, wpb, s);
        else if (src_grad(ln.src))
          mpvl::scan_band_batch_grad({(const ScanArgs*)desc, first, ln.nseg}, ln.src, ln.units, ln.LPL,
                                     ln.tau, wpb, s);
        else if (ln.src == SRC_CENSUS)
          mpvl::scan_band_batch({(const ScanArgs*)desc, first, ln.nseg}, ln.units, ln.LPL, ln.tau, wpb,
                                s);
        else
          mpvl::scan_band_batch_layered({(const ScanArgs*)desc, first, ln.nseg}, ln.src, ln.units,
                                        ln.LPL, ln.tau, wpb, s);
        break;
      }
      case mpv_batch_s::REDUCE: {
        mpvl::reduce_part_batch({(const RedArgs*)desc, first, ln.nseg}, ln.units, ln.stride, s);
        break;
      }
    }
    if (on_caux) {
      s = s_main;
      if (hipEventRecord(b->cjoin_ev[ln.level], b->caux) != hipSuccess) return MPV_ERR_DEVICE;
      cpend[ln.level] = true;
    } else if (s != s_main) {  // launched beside the previous launch: joined after both
      s = s_main;
      if (hipEventRecord(b->join_ev, b->aux) != hipSuccess || hipStreamWaitEvent(s, b->join_ev, 0) != hipSuccess)
        return MPV_ERR_DEVICE;
    }
  }
  for (int l = 0; l < MPV_MAX_LEVELS; ++l)  // a census no scan waited for (none planned so)
    if (cpend[l] && hipStreamWaitEvent(s, b->cjoin_ev[l], 0) != hipSuccess) return MPV_ERR_DEVICE;
  return launched();
}
}  // namespace

extern "C" {

mpv_status mpv_batch_run(mpv_batch b, hipStream_t s) {
  if (!b || !b->ws) return MPV_ERR_INVALID_ARG;
  return run_launches(b, b->launches, b->ws, s);
}

mpv_status mpv_batch_run_items(mpv_batch b, const int32_t* idx, int32_t n, hipStream_t s) {
  if (!b || !b->ws || !idx || n < 1 || n > (int32_t)b->pairs.size()) return MPV_ERR_INVALID_ARG;
  std::vector<char> seen(b->pairs.size(), 0);
  mpv_batch_s sub;
  sub.p = b->p;
  sub.table_bytes = b->table_bytes;
  for (int i = 0; i < n; ++i) {
    if (idx[i] < 0 || idx[i] >= (int32_t)b->pairs.size() || seen[idx[i]]) return MPV_ERR_INVALID_ARG;
    seen[idx[i]] = 1;
    sub.pairs.push_back(b->pairs[idx[i]]);  // keeps its workspace region (pr.off)
  }
  TableBuilder tb;
  plan_batch(sub, b->ws, tb);
  if (align_up(tb.bytes.size()) > b->table_bytes) return MPV_ERR_WORKSPACE;  // cannot happen: a subset
  if (!b->stage) {
    if (hipHostMalloc((void**)&b->stage, (size_t)mpv_batch_s::kStage * b->table_bytes) != hipSuccess) {
      b->stage = nullptr;
      return MPV_ERR_DEVICE;
    }
    for (int k = 0; k < mpv_batch_s::kStage; ++k)
      if (hipEventCreateWithFlags(&b->stage_ev[k], hipEventDisableTiming) != hipSuccess) return MPV_ERR_DEVICE;
  }
  const int k = b->stage_next;
  b->stage_next = (k + 1) % mpv_batch_s::kStage;
  // this staging entry was last uploaded kStage runs ago: wait until that copy has read it
  if (hipEventSynchronize(b->stage_ev[k]) != hipSuccess) return MPV_ERR_DEVICE;
  uint8_t* st = b->stage + (size_t)k * b->table_bytes;
  std::memcpy(st, tb.bytes.data(), tb.bytes.size());
  uint8_t* area = b->ws + b->table_bytes;
  if (hipMemcpyAsync(area, st, tb.bytes.size(), hipMemcpyHostToDevice, s) != hipSuccess) return MPV_ERR_DEVICE;
  if (hipEventRecord(b->stage_ev[k], s) != hipSuccess) return MPV_ERR_DEVICE;
  b->sub_launches = std::move(sub.launches);
  return run_launches(b, b->sub_launches, area, s);
}

mpv_status mpv_batch_run_graph(mpv_batch b, hipStream_t s) {
  if (!b || !b->ws) return MPV_ERR_INVALID_ARG;
  if (!b->exec) {
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return MPV_ERR_DEVICE;
    mpv_status st = MPV_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      st = MPV_ERR_DEVICE;
    } else {
      st = mpv_batch_run(b, cap);
      hipGraph_t g = nullptr;
      if (hipStreamEndCapture(cap, &g) != hipSuccess || !g) st = MPV_ERR_DEVICE;
      if (st == MPV_OK && hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        b->exec = nullptr;
        st = MPV_ERR_DEVICE;
      }
      b->graph = g;
    }
    (void)hipStreamDestroy(cap);
    if (st) return st;
  }
  return hipGraphLaunch(b->exec, s) == hipSuccess ? MPV_OK : MPV_ERR_DEVICE;
}

void mpv_batch_destroy(mpv_batch b) {
  if (!b) return;
  if (b->aux) {
    (void)hipStreamSynchronize(b->aux);
    (void)hipStreamDestroy(b->aux);
  }
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  if (b->join_ev) (void)hipEventDestroy(b->join_ev);
  if (b->caux) {
    (void)hipStreamSynchronize(b->caux);
    (void)hipStreamDestroy(b->caux);
  }
  if (b->cfork_ev) (void)hipEventDestroy(b->cfork_ev);
  for (int l = 0; l < MPV_MAX_LEVELS; ++l)
    if (b->cjoin_ev[l]) (void)hipEventDestroy(b->cjoin_ev[l]);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->stage) {
    for (int k = 0; k < mpv_batch_s::kStage; ++k)
      if (b->stage_ev[k]) {
        (void)hipEventSynchronize(b->stage_ev[k]);
        (void)hipEventDestroy(b->stage_ev[k]);
      }
    (void)hipHostFree(b->stage);
  }
  delete b;
}

// ---- learned band proposal: coarse level + features --------------------------------------
size_t mpv_lb_coarse_workspace_bytes(const mpv_params* p, int32_t W0, int32_t H0) {
  if (check_params(p, true) || p->merge != MPV_MERGE_SUM || p->grad_sigma != 0 ||
      p->data_term != MPV_DATA_CENSUS || W0 < 1 || H0 < 1 || W0 > MPV_MAX_WIDTH)
    return 0;
  const LevelWs lw = level_ws(p, W0, H0, nullptr, mpv_schedule{});
  return lw.fits ? lw.total : 0;
}

mpv_status mpv_lb_coarse(const mpv_params* p, const mpv_image* left0, const mpv_image* right0,
                         uint16_t* feat, int16_t* raw0, int16_t* disp0, void* workspace,
                         size_t workspace_bytes, hipStream_t stream) {
  mpv_status st = check_params(p, true);
  if (st) return st;
  if (p->merge != MPV_MERGE_SUM || p->grad_sigma != 0 || p->data_term != MPV_DATA_CENSUS)
    return MPV_ERR_UNSUPPORTED;
  if (!valid_image(left0) || !valid_image(right0) || !feat || !raw0 || !disp0)
    return MPV_ERR_INVALID_ARG;
  if (left0->width != right0->width || left0->height != right0->height) return MPV_ERR_INVALID_ARG;
  const int W = left0->width, H = left0->height;
  if (W > MPV_MAX_WIDTH) return MPV_ERR_INVALID_ARG;
  const mpv_schedule dflt{};
  const LevelWs lw = level_ws(p, W, H, nullptr, dflt);
  if (!lw.fits) return MPV_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < lw.total) return MPV_ERR_WORKSPACE;
  uint8_t* ws = (uint8_t*)workspace;
  st = run_level(p, left0->data, left0->pitch, right0->data, right0->pitch, W, H, nullptr, disp0,
                 nullptr, raw0, ws, 0, dflt, stream);
  if (st) return st;
  const float Z = (float)(p->num_paths * (24 + p->lambda * tau_eff(p->tau, p->num_disp)));
  mpvl::lb_features(ws + lw.part_off, (long long)H * W * lw.sc.capP, lw.sc.capP, p->num_paths,
                    p->num_disp, W, H, raw0, disp0, left0->data, left0->pitch, Z, feat, stream);
  return launched();
}

// ---- road profile (Section 3.5) -----------------------------------------------------------
static_assert(MPV_ROAD_MAX_HEIGHT == ROAD_MAX_HEIGHT, "road kernel LDS rows");
static_assert(MPV_MAX_DISP <= 256, "v- and u-disparity LDS histograms hold 256 disparities");
mpv_status mpv_vdisparity(const int16_t* disp, int32_t W, int32_t H, int32_t pitch, int32_t D,
                          uint32_t* hist, hipStream_t stream) {
  if (!disp || !hist || W < 1 || H < 1 || pitch < W || D < 1 || D > MPV_MAX_DISP) return MPV_ERR_INVALID_ARG;
  mpvl::vdisparity(disp, W, H, pitch, D, hist, stream);
  return launched();
}

mpv_status mpv_udisparity(const int16_t* disp, int32_t W, int32_t H, int32_t pitch, int32_t D,
                          uint32_t* hist, hipStream_t stream) {
  if (!disp || !hist || W < 1 || H < 1 || pitch < W || D < 1 || D > MPV_MAX_DISP) return MPV_ERR_INVALID_ARG;
  mpvl::udisparity(disp, W, H, pitch, D, hist, stream);
  return launched();
}

size_t mpv_road_workspace_bytes(int32_t D, int32_t H) {
  if (D < 1 || D > MPV_MAX_DISP || H < 1 || H > MPV_ROAD_MAX_HEIGHT) return 0;
  return align_up((size_t)D * H);
}

mpv_status mpv_road(const uint32_t* hist, int32_t D, int32_t H, int32_t eta, int16_t* path,
                    int32_t* energy, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!hist || !path || !energy || D < 1 || D > MPV_MAX_DISP || H < 1 || H > MPV_ROAD_MAX_HEIGHT ||
      eta < 2 || eta > 256)
    return MPV_ERR_INVALID_ARG;
  if (!workspace || workspace_bytes < mpv_road_workspace_bytes(D, H)) return MPV_ERR_WORKSPACE;
  mpvl::road(hist, D, H, eta, (uint8_t*)workspace, path, energy, stream);
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
