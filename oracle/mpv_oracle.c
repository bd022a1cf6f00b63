/*
 * CPU oracle for the multi-scale MPV (Multi-Path-Viterbi) stereo matcher.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no code, header, table or helper with the HIP path.
 *
 * Plain, slow, obviously correct integer code. Every energy is int64 and unnormalised:
 * it is the paper's node energy e(p,u) of the Viterbi recurrence (Section 3.2, eq. e(p,u))
 * with the data term replaced by a census/Hamming cost and the TV transition truncated:
 *
 *   C(x,y,d)  = popcount(cL(x,y) XOR cR(x-d,y)),  or 24 when x-d < 0
 *   L_r(p,d)  = C(p,d) + min_{d' in B(p-r)} [ L_r(p-r,d') + lambda * min(|d-d'|, tau) ]
 *   L_r(p,d)  = C(p,d) when p-r lies outside the image
 *
 * B(p) is the search band of pixel p: the disparities lo(p) .. lo(p)+len(p)-1, or the
 * full range [0, D) when no band is given. Disparities outside B(p) are absent nodes
 * (+infinity), which is how the paper's "virtual nodes" (Section 3.4) are read here.
 *
 * Two interchangeable transition modes:
 *   ORC_DEFINITION - the min over every predecessor node, O(|B|^2) per pixel, as the
 *                    paper sets L_u to all Viterbi nodes (Section 3.2).
 *   ORC_FAST       - the paper's O(2m) technique (Section 3.3, eqs. eq1-eq8): one
 *                    upward and one downward sweep over the disparity axis give the
 *                    untruncated L1 envelope; truncation adds one extra candidate
 *                    (the previous pixel's minimum plus lambda*tau). Exactly equal to
 *                    the definition.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <limits.h>

#define ORC_INF (INT64_MAX / 4)
#define ORC_DEFINITION 0
#define ORC_FAST 1

/* The eight scan directions r = (dx, dy), in the order of the paper's Multi-path
 * Viterbi table (Section 3.2, Table alg): left/right, up/down, the right-down/left-up
 * diagonal, the left-down/right-up diagonal. */
static const int DIR_DX[8] = {+1, -1, 0, 0, +1, -1, -1, +1};
static const int DIR_DY[8] = {0, 0, +1, -1, +1, -1, +1, -1};

int orc_dir_dx(int r) { return DIR_DX[r]; }
int orc_dir_dy(int r) { return DIR_DY[r]; }

/* Image pyramid (Section 3.4): each coarser layer halves both sides; a coarse pixel is
 * the rounded mean of its 2x2 block of finer pixels. */
void orc_downsample(const uint8_t *in, int W, int H, uint8_t *out)
{
    int w = W / 2, h = H / 2;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int s = in[(2 * y) * W + 2 * x] + in[(2 * y) * W + 2 * x + 1] +
                    in[(2 * y + 1) * W + 2 * x] + in[(2 * y + 1) * W + 2 * x + 1];
            out[y * w + x] = (uint8_t)((s + 2) >> 2);
        }
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Census transform over a 5x5 window: one bit per neighbour q != p, set when
 * I(q) < I(p); neighbour coordinates are clamped to the image. 24 bits. */
void orc_census5x5(const uint8_t *img, int W, int H, uint32_t *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            uint32_t c = 0;
            int bit = 0;
            int center = img[y * W + x];
            for (int dy = -2; dy <= 2; ++dy)
                for (int dx = -2; dx <= 2; ++dx) {
                    if (dx == 0 && dy == 0)
                        continue;
                    int v = img[clampi(y + dy, 0, H - 1) * W + clampi(x + dx, 0, W - 1)];
                    if (v < center)
                        c |= 1u << bit;
                    ++bit;
                }
            out[y * W + x] = c;
        }
}

static int popcount32(uint32_t v)
{
    int n = 0;
    while (v) {
        n += (int)(v & 1u);
        v >>= 1;
    }
    return n;
}

/* Band of pixel i: first disparity and number of disparities. */
static void band_of(const int16_t *lo, const uint8_t *len, int cap, long i, int *b0, int *bn)
{
    *b0 = lo ? lo[i] : 0;
    *bn = len ? len[i] : cap;
}

/* Matching cost volume [H][W][cap]; slot j holds disparity lo(p)+j. Slots past the
 * pixel's band length hold 0xFF. */
void orc_cost(const uint32_t *cl, const uint32_t *cr, int W, int H,
              const int16_t *lo, const uint8_t *len, int cap, uint8_t *cost)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            long i = (long)y * W + x;
            int b0, bn;
            band_of(lo, len, cap, i, &b0, &bn);
            for (int j = 0; j < cap; ++j) {
                uint8_t c = 0xFF;
                if (j < bn) {
                    int d = b0 + j;
                    c = (x - d >= 0) ? (uint8_t)popcount32(cl[i] ^ cr[i - d]) : 24;
                }
                cost[i * cap + j] = c;
            }
        }
}

static int64_t trans(int d, int dp, int lambda, int tau)
{
    int a = d > dp ? d - dp : dp - d;
    return (int64_t)lambda * (a < tau ? a : tau);
}

/* One pixel of the directed recurrence. prevL/prev band describe p-r; out is L(p, .). */
static void step_definition(const uint8_t *c, int b0, int bn, const int64_t *prevL, int q0, int qn,
                            int lambda, int tau, int64_t *out, int cap)
{
    for (int j = 0; j < cap; ++j)
        out[j] = ORC_INF;
    for (int j = 0; j < bn; ++j) {
        int d = b0 + j;
        int64_t best = ORC_INF;
        for (int k = 0; k < qn; ++k) {
            int64_t v = prevL[k] + trans(d, q0 + k, lambda, tau);
            if (v < best)
                best = v;
        }
        out[j] = (int64_t)c[j] + best;
    }
}

/* Section 3.3: instead of comparing every predecessor node, sweep the disparity axis
 * once upward and once downward. E_up(u) = min(E(p-1,u), E_up(u-1) + lambda) carries the
 * best predecessor below u, E_dn(u) = min(E(p-1,u), E_dn(u+1) + lambda) the best one above.
 * With truncation at tau, every predecessor further than tau costs the same lambda*tau,
 * so the previous minimum plus lambda*tau is the last candidate. scratch holds 3*D. */
static void step_fast(const uint8_t *c, int b0, int bn, const int64_t *prevL, int q0, int qn,
                      int lambda, int tau, int D, int64_t *out, int cap, int64_t *scratch)
{
    int64_t *A = scratch, *up = scratch + D, *dn = scratch + 2 * D;
    int64_t m = ORC_INF;
    for (int u = 0; u < D; ++u)
        A[u] = ORC_INF;
    for (int k = 0; k < qn; ++k) {
        A[q0 + k] = prevL[k];
        if (prevL[k] < m)
            m = prevL[k];
    }
    up[0] = A[0];
    for (int u = 1; u < D; ++u) {
        int64_t t = up[u - 1] + lambda;
        up[u] = A[u] < t ? A[u] : t;
    }
    dn[D - 1] = A[D - 1];
    for (int u = D - 2; u >= 0; --u) {
        int64_t t = dn[u + 1] + lambda;
        dn[u] = A[u] < t ? A[u] : t;
    }
    int64_t trunc = m + (int64_t)lambda * tau;
    for (int j = 0; j < cap; ++j)
        out[j] = ORC_INF;
    for (int j = 0; j < bn; ++j) {
        int u = b0 + j;
        int64_t h = up[u] < dn[u] ? up[u] : dn[u];
        if (trunc < h)
            h = trunc;
        out[j] = (int64_t)c[j] + h;
    }
}

/* L(p, .) for one pixel i whose predecessor along the path is q (q < 0: none). */
static void path_pixel(const uint8_t *cost, int D, const int16_t *lo, const uint8_t *len, int cap,
                       long i, long q, int lambda, int tau, int mode, int64_t *L, int64_t *scratch)
{
    int b0, bn;
    band_of(lo, len, cap, i, &b0, &bn);
    if (q < 0) {
        for (int j = 0; j < cap; ++j)
            L[i * cap + j] = j < bn ? (int64_t)cost[i * cap + j] : ORC_INF;
        return;
    }
    int q0, qn;
    band_of(lo, len, cap, q, &q0, &qn);
    if (mode == ORC_DEFINITION)
        step_definition(cost + i * cap, b0, bn, L + q * cap, q0, qn, lambda, tau, L + i * cap, cap);
    else
        step_fast(cost + i * cap, b0, bn, L + q * cap, q0, qn, lambda, tau, D, L + i * cap, cap,
                  scratch);
}

/* Energies of one directed path r over the whole image, L[H][W][cap].
 * Pixels are visited in an order where p-r always comes first. A horizontal path is a
 * set of independent rows (done in parallel); for the other directions every pixel of
 * a row depends only on the previous row in scan order, so a row is done in parallel
 * after the one before it. Returns 0, or -1 on bad arguments. */
int orc_path(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
             int cap, int r, int lambda, int tau, int mode, int64_t *L)
{
    if (r < 0 || r > 7 || W <= 0 || H <= 0 || cap <= 0 || D <= 0)
        return -1;
    int dx = DIR_DX[r], dy = DIR_DY[r];
    if (dy == 0) {
#pragma omp parallel
        {
            int64_t *scratch = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)D);
#pragma omp for schedule(static)
            for (int y = 0; y < H; ++y)
                for (int s = 0; s < W; ++s) {
                    int x = dx > 0 ? s : W - 1 - s;
                    int px = x - dx;
                    long q = (px < 0 || px >= W) ? -1 : (long)y * W + px;
                    path_pixel(cost, D, lo, len, cap, (long)y * W + x, q, lambda, tau, mode, L,
                               scratch);
                }
            free(scratch);
        }
        return 0;
    }
    for (int t = 0; t < H; ++t) {
        int y = dy > 0 ? t : H - 1 - t;
        int py = y - dy;
#pragma omp parallel
        {
            int64_t *scratch = (int64_t *)malloc(sizeof(int64_t) * 3 * (size_t)D);
#pragma omp for schedule(static)
            for (int x = 0; x < W; ++x) {
                int px = x - dx;
                long q = (py < 0 || py >= H || px < 0 || px >= W) ? -1 : (long)py * W + px;
                path_pixel(cost, D, lo, len, cap, (long)y * W + x, q, lambda, tau, mode, L,
                           scratch);
            }
            free(scratch);
        }
    }
    return 0;
}

/* Sum of the directed-path energies: S(p,d) = sum over the selected paths of L_r(p,d).
 * The selected paths are the first num_paths directions, further restricted to the bits
 * of path_mask when it is non-zero. Lscratch holds one [H][W][cap] int64 volume; when
 * per_path is non-NULL, path r's energies are also copied to per_path + r*H*W*cap. */
int orc_aggregate(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                  int cap, int num_paths, uint32_t path_mask, int lambda, int tau, int mode,
                  int64_t *S, int64_t *Lscratch, int64_t *per_path)
{
    long n = (long)W * H * cap;
    if (num_paths < 1 || num_paths > 8)
        return -1;
    for (long i = 0; i < n; ++i)
        S[i] = 0;
    for (int r = 0; r < num_paths; ++r) {
        if (path_mask && !(path_mask & (1u << r)))
            continue;
        int rc = orc_path(cost, W, H, D, lo, len, cap, r, lambda, tau, mode, Lscratch);
        if (rc)
            return rc;
        for (long i = 0; i < n; ++i) {
            if (Lscratch[i] >= ORC_INF || S[i] >= ORC_INF)
                S[i] = ORC_INF;
            else
                S[i] += Lscratch[i];
        }
        if (per_path)
            memcpy(per_path + (long)r * n, Lscratch, sizeof(int64_t) * (size_t)n);
    }
    return 0;
}

/* Winner-take-all and left-right check.
 *   dl(p)   = the smallest in-band d minimising S(p,d)                     (eq. viterbi)
 *   S'(p,d) = S(p,d) - min_d S(p,d)
 *   dr(x,y) = the largest d minimising S'(x+d,y,d) over the d with x+d < W and
 *             d in B(x+d,y); -1 when no such d exists. Every left pixel has S' = 0 at
 *             its own winner, so zero ties are common where several left pixels land on
 *             one right pixel; of those the one with the larger disparity is the nearer
 *             surface, the one the right camera sees.
 *   out(p)  = dl(p) when x-dl >= 0, dr(x-dl,y) >= 0 and |dl - dr(x-dl,y)| <= lr_max_diff,
 *             else -1; lr_max_diff < 0 disables the check (out = dl).
 * Any of dl/dr/out may be NULL except that out needs dl and dr internally. */
void orc_wta_lr(const int64_t *S, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                int cap, int lr_max_diff, int16_t *dl_out, int16_t *dr_out, int16_t *out)
{
    long npx = (long)W * H;
    int16_t *dl = (int16_t *)malloc(sizeof(int16_t) * (size_t)npx);
    int16_t *dr = (int16_t *)malloc(sizeof(int16_t) * (size_t)npx);
    int64_t *smin = (int64_t *)malloc(sizeof(int64_t) * (size_t)npx);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < npx; ++i) {
        int b0, bn;
        band_of(lo, len, cap, i, &b0, &bn);
        int64_t best = ORC_INF;
        int arg = -1;
        for (int j = 0; j < bn; ++j)
            if (S[i * cap + j] < best) {
                best = S[i * cap + j];
                arg = b0 + j;
            }
        dl[i] = (int16_t)arg;
        smin[i] = best;
    }
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t best = ORC_INF;
            int arg = -1;
            for (int d = 0; d < D && x + d < W; ++d) {
                long q = (long)y * W + x + d;
                int b0, bn;
                band_of(lo, len, cap, q, &b0, &bn);
                if (d < b0 || d >= b0 + bn)
                    continue;
                int64_t v = S[q * cap + (d - b0)] - smin[q];
                if (v <= best) {
                    best = v;
                    arg = d;
                }
            }
            dr[(long)y * W + x] = (int16_t)arg;
        }
    if (out) {
#pragma omp parallel for schedule(static)
        for (long i = 0; i < npx; ++i) {
            int x = (int)(i % W);
            int d = dl[i];
            int16_t o = (int16_t)d;
            if (lr_max_diff >= 0) {
                o = -1;
                if (d >= 0 && x - d >= 0) {
                    int r = dr[i - d];
                    int diff = r > d ? r - d : d - r;
                    if (r >= 0 && diff <= lr_max_diff)
                        o = (int16_t)d;
                }
            }
            out[i] = o;
        }
    }
    if (dl_out)
        memcpy(dl_out, dl, sizeof(int16_t) * (size_t)npx);
    if (dr_out)
        memcpy(dr_out, dr, sizeof(int16_t) * (size_t)npx);
    free(dl);
    free(dr);
    free(smin);
}

/* Coarse-to-fine band (Section 3.4: the coarser layer's disparity, transformed by the
 * sampling rate, seeds the search of the next layer). The center is twice the coarse
 * raw WTA disparity of the parent pixel (nearest upsampling, clamped to the coarse
 * image); the band is cap = min(2R+1, Dl) disparities starting at
 * lo = clamp(center - R, 0, Dl - cap). Returns cap. */
int orc_propagate(const int16_t *dl_coarse, int Wc, int Hc, int W, int H, int Dl, int R, int16_t *lo)
{
    int cap = 2 * R + 1 < Dl ? 2 * R + 1 : Dl;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int cx = x / 2 < Wc - 1 ? x / 2 : Wc - 1;
            int cy = y / 2 < Hc - 1 ? y / 2 : Hc - 1;
            int c = 2 * dl_coarse[cy * Wc + cx];
            lo[(long)y * W + x] = (int16_t)clampi(c - R, 0, Dl - cap);
        }
    return cap;
}
