// Banded scans with one scan line per lane (directions with dy != 0), instantiated only in
// kern_band_lines.hip.
#pragma once
#include "kernels.hpp"

namespace mpvk {

// ---------------------------------------------------------------------------------------
// Banded scan with one line per lane, for directions that cross image rows (dy != 0).
//
// Line u of direction (dx, dy) is at x = u + dx*g in scan row g (image row g going down,
// H-1-g going up); u runs over -(H-1)..W-1 (dx = +1), 0..W+H-2 (dx = -1) or 0..W-1
// (dx = 0), and line u is live in the scan rows where x lies inside the image, so it starts
// where p - r leaves the image, as the lines of the lane-group layout do. A wave holds 64
// neighbouring lines and walks their rows together: at every step its loads and stores touch
// consecutive pixels of one image row. A lane keeps its pixel's CAP band energies in
// registers. The min over predecessors (Section 3.3) is built from two linear sweeps along
// the band, E(i) = min(P(i), E(i-1) + lambda) and back, capped at lambda*tau: a predecessor
// at distance tau or more costs lambda*tau, so letting the sweeps run past tau-1 changes
// nothing. The envelope, with tau-1 extension slots on each side, goes to the lane's LDS row,
// and the new pixel's band reads it back at its offset lo(p) - lo(p-r); slots beyond the
// extension hold lambda*tau. A lane's energies stay zero until its line starts, and the
// line's first pixel reads them at offset 0: no transition term.
// Needs fixed-length bands with lo in [0, D-CAP] (the pyramid's own bands) and
// 24 + lambda*tau <= 255, so that every normalised energy is its own partial byte. Its
// levels use 12 partial slots per pixel (capP = 12): 12-byte stores of consecutive pixels
// (and 12-byte loads in the reduce) cover whole cache lines with a quarter fewer bytes than
// the 16-slot pitch of the lane groups. P6: where 24 + lambda*tau <= 63 every normalised
// energy fits six bits, and a pixel's slots go in 8 bytes instead (PART6_PITCH).
// ---------------------------------------------------------------------------------------
template <int CAP, int TAU>
struct LaneRow {
  static constexpr int M = TAU - 1;                 // extension slots on each side
  static constexpr int W0 = CAP;                    // first written entry (lambda*tau below)
  static constexpr int Q0 = W0 + M;                 // entry of the band's slot 0
  static constexpr int NW = CAP + 2 * M;            // entries written per step
  static constexpr int ENT = W0 + 2 * M + 2 * CAP;  // entries a read can reach
  static constexpr int DW = (ENT & 1) ? ENT : ENT + 1;  // odd: lanes' rows on distinct banks
};

__device__ __forceinline__ int wave_min_s(int v) { return -wave_max_s(-v); }

typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));

template <int CAP, int TAU, bool P6>
__device__ __forceinline__ void scan_lane_wave(const ScanArgs& a, const ScanArgs& tab, int unit) {
  using RW = LaneRow<CAP, TAU>;
  constexpr int M = RW::M;
  constexpr int LPF = 8;  // steps between a pixel's band-start load and its use
  constexpr int CPF = 2;  // steps between a pixel's census loads and their use
  constexpr int CH = 8;  // steps per chunk (one fast/slow decision)
  static_assert(LPF > CPF && CH % LPF == 0 && CH % CPF == 0, "rings divide the chunk");
  static_assert(CAP >= 1 && CAP <= (P6 ? PART6_SLOTS : 12), "a pixel's partials are one slot group");
  constexpr uint32_t PITCH = P6 ? PART6_PITCH : 12;
  __shared__ uint32_t lds_rows[4 * 64 * RW::DW];
  const int lane = lane_id();
  uint32_t* const row = lds_rows + (size_t)threadIdx.x * RW::DW;  // blockDim <= 256

  int ri = 0;
  while (ri + 1 < tab.ndir && unit >= tab.gprefix[ri + 1]) ++ri;
  const int r = tab.dir[ri];
  const int dx = c_dx[r], dy = c_dy[r];
  const int W = a.W, H = a.H;
  const int nl = dx == 0 ? W : W + H - 1;
  const int ib = (unit - tab.gprefix[ri]) * 64;  // first line of the wave
  const int u0 = ib + (dx > 0 ? -(H - 1) : 0);   // u of lane 0
  const int u = u0 + lane;
  int g0 = H, g1 = 0;  // scan rows [g0, g1) of this lane's line (empty past the last line)
  if (ib + lane < nl) {
    if (dx == 0) {
      g0 = 0;
      g1 = H;
    } else if (dx > 0) {
      g0 = max(0, -u);
      g1 = min(H, W - u);
    } else {
      g0 = max(0, u - W + 1);
      g1 = min(H, u + 1);
    }
  }
  const int gb = wave_min_s(g0), ge = wave_max_s(g1);
  if (gb >= ge) return;

  const uint32_t lam = (uint32_t)a.lambda;
  const uint32_t lt = (uint32_t)(a.lambda * a.tau);
  const int bmax = a.D - CAP;
  // the row: lambda*tau outside the slots written by every step
#pragma unroll
  for (int e = 0; e < RW::DW; ++e) row[e] = lt;

  uint8_t* const part = a.part + (long long)(a.dir_base + ri) * a.part_stride;
  const rsrc_t rpart = make_rsrc(part);
  const rsrc_t rcl = make_rsrc(a.cl);
  const rsrc_t rcr = make_rsrc(a.cr);
  const rsrc_t rlo = make_rsrc(a.lo);
  auto yat = [&](int g) { return dy > 0 ? g : H - 1 - g; };
  // lane-constant parts of the offsets; the fast path adds the row's uniform part (lane 0's
  // pixel) as the scalar offset
  const uint32_t vcl = (uint32_t)(lane + a.cmargin) << 2;
  const int vcr = (lane + a.cmargin - (CAP - 1)) << 2;  // >= 4*(D + 64) - 4*(CAP-1) > 4*bmax
  const uint32_t vlo = (uint32_t)lane << 1;
  const uint32_t vpart = (uint32_t)lane * PITCH;

  // prefetch rings: band starts of steps g .. g+LPF-1, census of steps g .. g+CPF-1
  int b0q[LPF];
  uint32_t clq[CPF], crq[CPF][CAP];
  // per-lane (clamped) pixel and census offsets of scan row g, for the slow path
  auto pix_at = [&](int g, int& p, int& c, int& x) {
    const int gc = min(max(g, 0), H - 1);
    x = u + dx * gc;
    const int xc = min(max(x, 0), W - 1);
    const int y = yat(gc);
    p = y * W + xc;
    c = y * a.cpitch + a.cmargin + xc;
  };
  auto load_lo_slow = [&](int g) -> int {
    int p, c, x;
    pix_at(g, p, c, x);
    return (int)(short)buf_ld16(rlo, (uint32_t)p << 1, 0u);
  };
  auto load_cen_slow = [&](int g, int b0, uint32_t& cl, uint32_t (&cr)[CAP]) {
    int p, c, x;
    pix_at(g, p, c, x);
    cl = buf_ld32(rcl, (uint32_t)c << 2, 0u);
    const uint32_t vo = (uint32_t)(c - b0 - (CAP - 1)) << 2;  // census margin >= D + 64
#pragma unroll
    for (int k = 0; k < CAP; ++k) cr[CAP - 1 - k] = buf_ld32(rcr, vo + 4 * k, 0u);
  };
#pragma unroll
  for (int q = 0; q < LPF; ++q) b0q[q] = load_lo_slow(gb + q);
#pragma unroll
  for (int q = 0; q < CPF; ++q) {
    b0q[q] = min(max(b0q[q], 0), bmax);
    load_cen_slow(gb + q, b0q[q], clq[q], crq[q]);
  }

  uint32_t P[CAP];
#pragma unroll
  for (int i = 0; i < CAP; ++i) P[i] = 0;
  int lo_prev = 0;

  auto step = [&](auto kc, auto fc, int g) {
    constexpr int k = decltype(kc)::value;
    constexpr bool FAST = decltype(fc)::value;
    constexpr int s2 = k % LPF, s1 = k % CPF, sn = (k + CPF) % LPF;
    const int b0 = b0q[s2];
    const uint32_t cl = clq[s1];
    uint32_t cr[CAP];
#pragma unroll
    for (int j = 0; j < CAP; ++j) cr[j] = crq[s1][j];
    // loads: census of step g + CPF (its band start arrived LPF - CPF steps ago), band start
    // of step g + LPF
    {
      const int bn = min(max(b0q[sn], 0), bmax);
      b0q[sn] = bn;
      if constexpr (FAST) {
        const int gq = g + CPF, gl = g + LPF;
        const uint32_t cu = (uint32_t)(yat(gq) * a.cpitch + u0 + dx * gq) << 2;
        clq[s1] = buf_ld32(rcl, vcl, cu);
        const uint32_t vo = (uint32_t)(vcr - 4 * bn);
#pragma unroll
        for (int q = 0; q < CAP; ++q) crq[s1][CAP - 1 - q] = buf_ld32(rcr, vo + 4 * q, cu);
        b0q[s2] = (int)(short)buf_ld16(rlo, vlo, (uint32_t)(yat(gl) * W + u0 + dx * gl) << 1);
      } else {
        load_cen_slow(g + CPF, bn, clq[s1], crq[s1]);
        b0q[s2] = load_lo_slow(g + LPF);
      }
    }
    // envelope of the previous pixel's band, with M extension slots on each side
    uint32_t A[CAP], B[CAP];
    A[0] = P[0];
#pragma unroll
    for (int i = 1; i < CAP; ++i) A[i] = min(P[i], A[i - 1] + lam);
    B[CAP - 1] = P[CAP - 1];
#pragma unroll
    for (int i = CAP - 2; i >= 0; --i) B[i] = min(P[i], B[i + 1] + lam);
    uint32_t* const wr = row + RW::W0;
#pragma unroll
    for (int e = 1; e <= M; ++e) wr[M - e] = min(B[0] + e * lam, lt);
#pragma unroll
    for (int i = 0; i < CAP; ++i) wr[M + i] = min(min(A[i], B[i]), lt);
#pragma unroll
    for (int e = 1; e <= M; ++e) wr[M + CAP - 1 + e] = min(A[CAP - 1] + e * lam, lt);
    // this pixel's band in the previous pixel's frame; a line's first pixel reads the band
    // itself, all zeros (a lane's energies stay zero until its line starts)
    int sidx = min(max(b0 - lo_prev, -(CAP + M)), CAP + M);
    bool live = true;
    int xl = 0;
    if constexpr (!FAST) {
      live = g >= g0 && g < g1;
      if (g == g0) sidx = 0;
      xl = u + dx * g - b0;  // candidates j > xl have x - d < 0
    }
    const uint32_t* const rd = row + RW::Q0 + sidx;
    uint32_t L[CAP];
#pragma unroll
    for (int j = 0; j < CAP; ++j) {
      uint32_t h = cl ^ cr[j];
      if constexpr (!FAST) h = j > xl ? 0xFFFFFFu : h;  // outside the right image: cost 24
      L[j] = (uint32_t)__popc(h) + rd[j];
    }
    uint32_t m = L[0];
#pragma unroll
    for (int j = 1; j < CAP; ++j) m = min(m, L[j]);
#pragma unroll
    for (int j = 0; j < CAP; ++j) P[j] = L[j] - m;
    if constexpr (!FAST) {
      if (g < g0) {
#pragma unroll
        for (int j = 0; j < CAP; ++j) P[j] = 0;
      }
    }
    // the pixel's partials (offsets in the vector register: a 16-byte buffer store with a
    // scalar offset has been seen to store the next instruction's result in its upper half,
    // and the compiler models that hazard only for stores without a scalar offset register)
    const uint32_t po = FAST ? vpart + (uint32_t)(yat(g) * W + u0 + dx * g) * PITCH : 0u;
    if constexpr (P6) {
      // six-bit fields (every normalised energy is at most 24 + lambda*tau <= 63)
      u32x2 w = {0u, 0u};
#pragma unroll
      for (int i = 0; i < CAP; ++i) w[i / 5] |= P[i] << (6 * (i % 5));
      if constexpr (FAST) {
        __builtin_amdgcn_raw_buffer_store_b64(w, rpart, (int)po, 0, kPartStorePolicy);
      } else if (live) {
        int p, c, x;
        pix_at(g, p, c, x);
        __builtin_amdgcn_raw_buffer_store_b64(w, rpart, (int)((uint32_t)p * PITCH), 0, kPartStorePolicy);
      }
    } else {
      // bytes (every normalised energy is at most 24 + lambda*tau <= 255), 255 past CAP
      u32x3 w = {0u, 0u, 0u};
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        uint32_t v = 0;
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) v |= (4 * q + bb < CAP ? P[min(4 * q + bb, CAP - 1)] : 0xFFu) << (8 * bb);
        w[q] = v;
      }
      if constexpr (FAST) {
        __builtin_amdgcn_raw_buffer_store_b96(w, rpart, (int)po, 0, kPartStorePolicy);
      } else if (live) {
        int p, c, x;
        pix_at(g, p, c, x);
        __builtin_amdgcn_raw_buffer_store_b96(w, rpart, (int)((uint32_t)p * PITCH), 0, kPartStorePolicy);
      }
    }
    lo_prev = b0;
  };

  for (int g = gb; g < ge; g += CH) {
    // fast chunk: every lane's line covers the chunk and its loads, none starts in it, and
    // every candidate x - d of the chunk lies inside the right image
    const int xmin = u + dx * (dx > 0 ? g : g + CH - 1);
    const bool fast = wave_all(g0 < g && g + CH + LPF <= g1 && xmin >= a.D - 1);
    if (fast) {
      static_for<CH>([&](auto kc) { step(kc, std::true_type{}, g + decltype(kc)::value); });
    } else {
      static_for<CH>([&](auto kc) { step(kc, std::false_type{}, g + decltype(kc)::value); });
    }
  }
}

// Batched banded scans with one line per lane; P6: six-bit partial slots.
template <int TAU, int CAP, bool P6>
__global__ __launch_bounds__(256) void k_scan_lane_batch(Batch<ScanArgs> b) {
  const int u = wave_unit();
  if (u >= b.first[b.nseg]) return;
  const int s = batch_find(b.first, b.nseg, u);
  const ScanArgs a = b.desc[s];  // private copy, as above
  scan_lane_wave<CAP, TAU, P6>(a, b.desc[s], u - b.first[s]);
}

}  // namespace mpvk
