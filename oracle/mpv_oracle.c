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
 *
 * Two ways of merging the directed paths:
 *   orc_aggregate  - the sum S(p,d) = sum_r L_r(p,d) over the selected paths.
 *   orc_layered    - the paper's hierarchical merge (Section 3.2, Table alg): four layers
 *                    of opposite direction pairs, each pair merged per node (min for the
 *                    horizontal layer, the mean for the others) and passed to the next
 *                    layer as its data term, so the recurrence also runs over int64 data.
 *
 * Transition weight: lambda, or (the *_g variants with an image and sigma > 0) the
 * gradient-weighted TV of eq. EU, lambda * exp(-|G|) with G the intensity difference of
 * the left image between the two consecutive path pixels divided by sigma, rounded to the
 * nearest integer (orc_grad_weight).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <limits.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

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

/* Threads of the OpenMP loops (n >= 1); returns the previous maximum (1 without OpenMP). */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    int prev = omp_get_max_threads();
    if (n >= 1)
        omp_set_num_threads(n);
    return prev;
#else
    (void)n;
    return 1;
#endif
}

/* Gradient-weighted TV weight of eq. EU: round(lambda * exp(-g / sigma)) for an intensity
 * difference g >= 0 between consecutive path pixels; sigma <= 0 keeps lambda. */
int orc_grad_weight(int lambda, int sigma, int g)
{
    if (sigma <= 0)
        return lambda;
    return (int)floor((double)lambda * exp(-(double)g / (double)sigma) + 0.5);
}

/* Transition weight from disparity dp at p-r to d at p. up multiplies the weight of an
 * increase of disparity (dp < d); it is 1 except in the left-to-right pass of the layered
 * merge with the occlusion strategy (orc_layered). */
static int64_t trans(int d, int dp, int lambda, int tau, int up)
{
    int a = d > dp ? d - dp : dp - d;
    return (int64_t)(d > dp ? up : 1) * lambda * (a < tau ? a : tau);
}

/* One pixel of the directed recurrence. c is the pixel's data term over its band slots;
 * prevL/prev band describe p-r; out is L(p, .). */
static void step_definition(const int64_t *c, int b0, int bn, const int64_t *prevL, int q0, int qn,
                            int lambda, int tau, int up, int64_t *out, int cap)
{
    for (int j = 0; j < cap; ++j)
        out[j] = ORC_INF;
    for (int j = 0; j < bn; ++j) {
        int d = b0 + j;
        int64_t best = ORC_INF;
        for (int k = 0; k < qn; ++k) {
            int64_t v = prevL[k] + trans(d, q0 + k, lambda, tau, up);
            if (v < best)
                best = v;
        }
        out[j] = c[j] + best;
    }
}

/* Section 3.3: instead of comparing every predecessor node, sweep the disparity axis
 * once upward and once downward. E_up(u) = min(E(p-1,u), E_up(u-1) + up*lambda) carries
 * the best predecessor below u, E_dn(u) = min(E(p-1,u), E_dn(u+1) + lambda) the best one
 * above. With truncation at tau every predecessor at least tau below u costs up*lambda*tau
 * and every one at least tau above costs lambda*tau, so the minima of the predecessors at
 * or below u (plus up*lambda*tau) and at or above u (plus lambda*tau) are the last two
 * candidates; for up = 1 both reduce to the previous minimum plus lambda*tau.
 * scratch holds 5*D. */
static void step_fast(const int64_t *c, int b0, int bn, const int64_t *prevL, int q0, int qn,
                      int lambda, int tau, int up, int D, int64_t *out, int cap, int64_t *scratch)
{
    int64_t *A = scratch, *upE = scratch + D, *dnE = scratch + 2 * D;
    int64_t *pre = scratch + 3 * D, *suf = scratch + 4 * D;
    for (int u = 0; u < D; ++u)
        A[u] = ORC_INF;
    for (int k = 0; k < qn; ++k)
        A[q0 + k] = prevL[k];
    upE[0] = A[0];
    pre[0] = A[0];
    for (int u = 1; u < D; ++u) {
        int64_t t = upE[u - 1] + (int64_t)up * lambda;
        upE[u] = A[u] < t ? A[u] : t;
        pre[u] = A[u] < pre[u - 1] ? A[u] : pre[u - 1];
    }
    dnE[D - 1] = A[D - 1];
    suf[D - 1] = A[D - 1];
    for (int u = D - 2; u >= 0; --u) {
        int64_t t = dnE[u + 1] + lambda;
        dnE[u] = A[u] < t ? A[u] : t;
        suf[u] = A[u] < suf[u + 1] ? A[u] : suf[u + 1];
    }
    for (int j = 0; j < cap; ++j)
        out[j] = ORC_INF;
    for (int j = 0; j < bn; ++j) {
        int u = b0 + j;
        int64_t h = upE[u] < dnE[u] ? upE[u] : dnE[u];
        int64_t t1 = pre[u] + (int64_t)up * lambda * tau, t2 = suf[u] + (int64_t)lambda * tau;
        if (t1 < h)
            h = t1;
        if (t2 < h)
            h = t2;
        out[j] = c[j] + h;
    }
}

/* L(p, .) for one pixel i whose predecessor along the path is q (q < 0: none). */
static void path_pixel(const int64_t *data, int D, const int16_t *lo, const uint8_t *len, int cap,
                       long i, long q, int lambda, int tau, int up, const uint8_t *img, int sigma,
                       int mode, int64_t *L, int64_t *scratch)
{
    int b0, bn;
    band_of(lo, len, cap, i, &b0, &bn);
    if (q < 0) {
        for (int j = 0; j < cap; ++j)
            L[i * cap + j] = j < bn ? data[i * cap + j] : ORC_INF;
        return;
    }
    int q0, qn;
    band_of(lo, len, cap, q, &q0, &qn);
    if (img && sigma > 0) /* the weight of the edge q -> i (eq. EU) */
        lambda = orc_grad_weight(lambda, sigma, abs((int)img[i] - (int)img[q]));
    if (mode == ORC_DEFINITION)
        step_definition(data + i * cap, b0, bn, L + q * cap, q0, qn, lambda, tau, up, L + i * cap,
                        cap);
    else
        step_fast(data + i * cap, b0, bn, L + q * cap, q0, qn, lambda, tau, up, D, L + i * cap, cap,
                  scratch);
}

/* Energies of one directed path r over the whole image, L[H][W][cap], for an int64 data
 * term data[H][W][cap] (slot j of pixel p = disparity lo(p)+j).
 * Pixels are visited in an order where p-r always comes first. A horizontal path is a
 * set of independent rows (done in parallel); for the other directions every pixel of
 * a row depends only on the previous row in scan order, so a row is done in parallel
 * after the one before it. Returns 0, or -1 on bad arguments. */
static int path_run(const int64_t *data, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                    int cap, int r, int lambda, int tau, int up, const uint8_t *img, int sigma,
                    int mode, int64_t *L)
{
    if (r < 0 || r > 7 || W <= 0 || H <= 0 || cap <= 0 || D <= 0)
        return -1;
    int dx = DIR_DX[r], dy = DIR_DY[r];
    if (dy == 0) {
#pragma omp parallel
        {
            int64_t *scratch = (int64_t *)malloc(sizeof(int64_t) * 5 * (size_t)D);
#pragma omp for schedule(static)
            for (int y = 0; y < H; ++y)
                for (int s = 0; s < W; ++s) {
                    int x = dx > 0 ? s : W - 1 - s;
                    int px = x - dx;
                    long q = (px < 0 || px >= W) ? -1 : (long)y * W + px;
                    path_pixel(data, D, lo, len, cap, (long)y * W + x, q, lambda, tau, up, img, sigma,
                               mode, L, scratch);
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
            int64_t *scratch = (int64_t *)malloc(sizeof(int64_t) * 5 * (size_t)D);
#pragma omp for schedule(static)
            for (int x = 0; x < W; ++x) {
                int px = x - dx;
                long q = (py < 0 || py >= H || px < 0 || px >= W) ? -1 : (long)py * W + px;
                path_pixel(data, D, lo, len, cap, (long)y * W + x, q, lambda, tau, up, img, sigma,
                           mode, L, scratch);
            }
            free(scratch);
        }
    }
    return 0;
}

/* Energies of one directed path r over the matching cost volume cost[H][W][cap]; img
 * (the left image [H][W]) and sigma > 0 select the gradient-weighted transition. */
int orc_path_g(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
               int cap, int r, int lambda, int tau, const uint8_t *img, int sigma, int mode,
               int64_t *L)
{
    long n = (long)W * H * cap;
    if (W <= 0 || H <= 0 || cap <= 0)
        return -1;
    int64_t *data = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (long i = 0; i < n; ++i)
        data[i] = cost[i];
    int rc = path_run(data, W, H, D, lo, len, cap, r, lambda, tau, 1, img, sigma, mode, L);
    free(data);
    return rc;
}

int orc_path(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
             int cap, int r, int lambda, int tau, int mode, int64_t *L)
{
    return orc_path_g(cost, W, H, D, lo, len, cap, r, lambda, tau, NULL, 0, mode, L);
}

/* Sum of the directed-path energies: S(p,d) = sum over the selected paths of L_r(p,d).
 * The selected paths are the first num_paths directions, further restricted to the bits
 * of path_mask when it is non-zero. Lscratch holds one [H][W][cap] int64 volume; when
 * per_path is non-NULL, path r's energies are also copied to per_path + r*H*W*cap. */
int orc_aggregate_g(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                    int cap, int num_paths, uint32_t path_mask, int lambda, int tau,
                    const uint8_t *img, int sigma, int mode, int64_t *S, int64_t *Lscratch,
                    int64_t *per_path)
{
    long n = (long)W * H * cap;
    if (num_paths < 1 || num_paths > 8)
        return -1;
    for (long i = 0; i < n; ++i)
        S[i] = 0;
    for (int r = 0; r < num_paths; ++r) {
        if (path_mask && !(path_mask & (1u << r)))
            continue;
        int rc = orc_path_g(cost, W, H, D, lo, len, cap, r, lambda, tau, img, sigma, mode, Lscratch);
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

int orc_aggregate(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                  int cap, int num_paths, uint32_t path_mask, int lambda, int tau, int mode,
                  int64_t *S, int64_t *Lscratch, int64_t *per_path)
{
    return orc_aggregate_g(cost, W, H, D, lo, len, cap, num_paths, path_mask, lambda, tau, NULL, 0,
                           mode, S, Lscratch, per_path);
}

/* Layered merge of bi-directional paths (Section 3.2, the hierarchical merging of the
 * paths and Table alg). Layer k = 0 .. num_layers-1 runs the two opposite directions 2k
 * and 2k+1 of the table's order (left/right, up/down, the two diagonals) over a data
 * term: the matching cost for the first layer, the previous layer's merged energy for the
 * others (the current layer's node energies seed the next layer). Each direction's
 * energies are taken relative to the pixel's minimum over its band,
 *   Fh(p,d) = F(p,d) - min_d' F(p,d'),  Bh(p,d) = B(p,d) - min_d' B(p,d'),
 * and merged per node: the horizontal layer keeps min(Fh, Bh) (sharpens edges), the
 * others floor((Fh + Bh) / 2) (the mean, removes noise). occ != 0 applies the example
 * strategy for occluded areas: the left-to-right pass (direction 0) pays twice the
 * transition weight when the disparity increases. M[H][W][cap] receives the last layer's
 * merged energies (absent slots ORC_INF); per_layer, when non-NULL, receives layer k's at
 * per_layer + k*H*W*cap. Returns 0, or -1 on bad arguments. */
int orc_layered_g(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                  int cap, int num_layers, int lambda, int tau, int occ, const uint8_t *img,
                  int sigma, int mode, int64_t *M, int64_t *per_layer)
{
    long npx = (long)W * H, n = npx * cap;
    if (num_layers < 1 || num_layers > 4 || W <= 0 || H <= 0 || cap <= 0)
        return -1;
    int64_t *data = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *F = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *B = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (long i = 0; i < n; ++i)
        data[i] = cost[i];
    int rc = 0;
    for (int k = 0; k < num_layers && rc == 0; ++k) {
        rc = path_run(data, W, H, D, lo, len, cap, 2 * k, lambda, tau, (occ && k == 0) ? 2 : 1,
                      img, sigma, mode, F);
        if (rc == 0)
            rc = path_run(data, W, H, D, lo, len, cap, 2 * k + 1, lambda, tau, 1, img, sigma, mode, B);
        if (rc)
            break;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < npx; ++i) {
            int b0, bn;
            band_of(lo, len, cap, i, &b0, &bn);
            int64_t fm = ORC_INF, bm = ORC_INF;
            for (int j = 0; j < bn; ++j) {
                if (F[i * cap + j] < fm)
                    fm = F[i * cap + j];
                if (B[i * cap + j] < bm)
                    bm = B[i * cap + j];
            }
            for (int j = 0; j < cap; ++j) {
                int64_t v = ORC_INF;
                if (j < bn) {
                    int64_t f = F[i * cap + j] - fm, b = B[i * cap + j] - bm;
                    v = k == 0 ? (f < b ? f : b) : (f + b) / 2;
                }
                M[i * cap + j] = v;
            }
        }
        if (per_layer)
            memcpy(per_layer + (long)k * n, M, sizeof(int64_t) * (size_t)n);
        memcpy(data, M, sizeof(int64_t) * (size_t)n);
    }
    free(data);
    free(F);
    free(B);
    return rc;
}

int orc_layered(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                int cap, int num_layers, int lambda, int tau, int occ, int mode, int64_t *M,
                int64_t *per_layer)
{
    return orc_layered_g(cost, W, H, D, lo, len, cap, num_layers, lambda, tau, occ, NULL, 0, mode,
                         M, per_layer);
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

/* The paper's own propagation (Section 3.4), intermediate layer. Only the pixels sampled
 * from the coarser layer carry an initial value (twice the coarser raw WTA: the values are
 * transformed by the sampling rate); the layer is split into blocks of block x block pixels
 * and every pixel of a block searches around the block's mode of those initial values.
 * The initial values of a block are those of the distinct parents of its pixels (pixel
 * (x, y) has parent (min(x/2, Wc-1), min(y/2, Hc-1)), so border blocks past the coarse
 * image still see their nearest parents); the mode is the most frequent value, the
 * smallest one on ties. Band: cap = min(2R+1, Dl) disparities from
 * lo = clamp(2*mode - R, 0, Dl - cap). Returns cap. */
int orc_propagate_block(const int16_t *dl_coarse, int Wc, int Hc, int W, int H, int Dl, int R,
                        int block, int16_t *lo)
{
    int cap = 2 * R + 1 < Dl ? 2 * R + 1 : Dl;
    for (int by0 = 0; by0 < H; by0 += block)
        for (int bx0 = 0; bx0 < W; bx0 += block) {
            int bx1 = bx0 + block < W ? bx0 + block : W;
            int by1 = by0 + block < H ? by0 + block : H;
            int cx0 = clampi(bx0 / 2, 0, Wc - 1), cx1 = clampi((bx1 - 1) / 2, 0, Wc - 1);
            int cy0 = clampi(by0 / 2, 0, Hc - 1), cy1 = clampi((by1 - 1) / 2, 0, Hc - 1);
            int best_v = 0, best_n = 0;
            for (int j = cy0; j <= cy1; ++j)
                for (int i = cx0; i <= cx1; ++i) {
                    int v = dl_coarse[j * Wc + i], n = 0;
                    for (int jj = cy0; jj <= cy1; ++jj)
                        for (int ii = cx0; ii <= cx1; ++ii)
                            n += dl_coarse[jj * Wc + ii] == v;
                    if (n > best_n || (n == best_n && v < best_v)) {
                        best_n = n;
                        best_v = v;
                    }
                }
            int16_t l = (int16_t)clampi(2 * best_v - R, 0, Dl - cap);
            for (int y = by0; y < by1; ++y)
                for (int x = bx0; x < bx1; ++x)
                    lo[(long)y * W + x] = l;
        }
    return cap;
}

/* The paper's own propagation (Section 3.4), last layer: every pixel is its own block.
 * The sampled pixels (2i, 2j) take twice the coarser raw WTA of (i, j); the others are
 * initialised by linear interpolation between the sampled pixels around them: midway
 * between two samples the mean of their values, at the centre of four samples the mean
 * of all four rounded half up (samples past the coarse image are clamped to its last
 * row/column). Band as in orc_propagate_block. Returns cap. */
int orc_propagate_interp(const int16_t *dl_coarse, int Wc, int Hc, int W, int H, int Dl, int R,
                         int16_t *lo)
{
    int cap = 2 * R + 1 < Dl ? 2 * R + 1 : Dl;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int i0 = clampi(x / 2, 0, Wc - 1), i1 = clampi(x / 2 + (x & 1), 0, Wc - 1);
            int j0 = clampi(y / 2, 0, Hc - 1), j1 = clampi(y / 2 + (y & 1), 0, Hc - 1);
            /* values of the (up to) four samples, each twice the coarse disparity */
            int s = 2 * dl_coarse[j0 * Wc + i0] + 2 * dl_coarse[j0 * Wc + i1] +
                    2 * dl_coarse[j1 * Wc + i0] + 2 * dl_coarse[j1 * Wc + i1];
            int c = (s + 2) >> 2;
            lo[(long)y * W + x] = (int16_t)clampi(c - R, 0, Dl - cap);
        }
    return cap;
}

/* SSIM data term (Section 3.2, eqs. components and ssim), following the structural
 * similarity index of the work the paper cites for it, with that work's constants:
 * K1 = 0.01, K2 = 0.03, L = 255 (8-bit pixels), C1 = (K1 L)^2, C2 = (K2 L)^2, C3 = C2/2 and
 * alpha = beta = gamma = 1. psi and phi are N x N = 5 x 5 patches (uniform weights) of the
 * left image around p and of the right image around p - (u, 0), coordinates clamped to the
 * image. With the means, (population) variances and covariance of the patches,
 *   l = (2 mu_psi mu_phi + C1) / (mu_psi^2 + mu_phi^2 + C1)
 *   c = (2 sigma_psi sigma_phi + C2) / (sigma_psi^2 + sigma_phi^2 + C2)
 *   s = (sigma_psiphi + C3) / (sigma_psi sigma_phi + C3)
 * (the printed c has mu^2 mu^2 in its denominator and the printed s is inverted; these are
 * the cited work's forms). Since C3 = C2/2, 2 sigma_psi sigma_phi + C2 = 2 (sigma_psi
 * sigma_phi + C3), so c s = (2 sigma_psiphi + C2) / (sigma_psi^2 + sigma_phi^2 + C2) exactly
 * and SSIM = l c s needs no square root. Every moment is a patch sum over n = 25 integer
 * pixels, and C1 = 65025 / 10^4, C2 = 585225 / 10^4 are exact decimals, so scaling all four
 * factors by n^2 10^4 makes SSIM an exact ratio of integers, num / den with den > 0.
 * The cost (eq. ssim) is (1 - SSIM) L' / 2 with the data-term scale L' = 24, the range of the
 * census cost, so the transition weights keep their meaning; it is rounded half up:
 *   cost = floor((24 (den - num) + den) / (2 den)),  0 <= cost <= 24,
 * in 128-bit integer arithmetic. A candidate with x - u < 0 costs 24. */
#define SSIM_Q 24
#define SSIM_SCALE 10000
#define SSIM_C1S 65025  /* (0.01 * 255)^2 * 10^4 */
#define SSIM_C2S 585225 /* (0.03 * 255)^2 * 10^4 */

/* Exact SSIM of two 25-pixel patches: num / den. */
void orc_ssim_ratio(const uint8_t *psi, const uint8_t *phi, __int128 *num, __int128 *den)
{
    const int64_t n = 25;
    int64_t A = 0, B = 0, AA = 0, BB = 0, AB = 0;
    for (int k = 0; k < 25; ++k) {
        A += psi[k];
        B += phi[k];
        AA += (int64_t)psi[k] * psi[k];
        BB += (int64_t)phi[k] * phi[k];
        AB += (int64_t)psi[k] * phi[k];
    }
    /* n^2 10^4 (2 mu_psi mu_phi + C1), n^2 10^4 (2 sigma_psiphi + C2),
       n^2 10^4 (mu_psi^2 + mu_phi^2 + C1), n^2 10^4 (sigma_psi^2 + sigma_phi^2 + C2) */
    int64_t f1 = 2 * SSIM_SCALE * A * B + SSIM_C1S * n * n;
    int64_t f2 = 2 * SSIM_SCALE * (n * AB - A * B) + SSIM_C2S * n * n;
    int64_t g1 = SSIM_SCALE * (A * A + B * B) + SSIM_C1S * n * n;
    int64_t g2 = SSIM_SCALE * (n * AA - A * A + n * BB - B * B) + SSIM_C2S * n * n;
    *num = (__int128)f1 * f2;
    *den = (__int128)g1 * g2;
}

/* SSIM as num / den in two 64-bit halves each (for callers without 128-bit integers). */
void orc_ssim_ratio_parts(const uint8_t *psi, const uint8_t *phi, int64_t *num_hi, uint64_t *num_lo,
                          int64_t *den_hi, uint64_t *den_lo)
{
    __int128 num, den;
    orc_ssim_ratio(psi, phi, &num, &den);
    *num_hi = (int64_t)(num >> 64);
    *num_lo = (uint64_t)num;
    *den_hi = (int64_t)(den >> 64);
    *den_lo = (uint64_t)den;
}

/* Quantised SSIM cost of two patches (eq. ssim), 0 .. 24. */
int orc_ssim_patch_cost(const uint8_t *psi, const uint8_t *phi)
{
    __int128 num, den;
    orc_ssim_ratio(psi, phi, &num, &den);
    return (int)((SSIM_Q * (den - num) + den) / (2 * den));
}

/* SSIM cost volume [H][W][cap] (slot j = disparity lo(p)+j; slots past the band 0xFF), the
 * SSIM counterpart of orc_cost. */
void orc_ssim_cost(const uint8_t *left, const uint8_t *right, int W, int H, const int16_t *lo,
                   const uint8_t *len, int cap, uint8_t *cost)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            long i = (long)y * W + x;
            int b0, bn;
            band_of(lo, len, cap, i, &b0, &bn);
            uint8_t psi[25], phi[25];
            int k = 0;
            for (int dy = -2; dy <= 2; ++dy)
                for (int dx = -2; dx <= 2; ++dx)
                    psi[k++] = left[clampi(y + dy, 0, H - 1) * W + clampi(x + dx, 0, W - 1)];
            for (int j = 0; j < cap; ++j) {
                uint8_t c = 0xFF;
                if (j < bn) {
                    int d = b0 + j;
                    if (x - d < 0) {
                        c = SSIM_Q;
                    } else {
                        k = 0;
                        for (int dy = -2; dy <= 2; ++dy)
                            for (int dx = -2; dx <= 2; ++dx)
                                phi[k++] = right[clampi(y + dy, 0, H - 1) * W + clampi(x - d + dx, 0, W - 1)];
                        c = (uint8_t)orc_ssim_patch_cost(psi, phi);
                    }
                }
                cost[i * cap + j] = c;
            }
        }
}
