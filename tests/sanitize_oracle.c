/* Test driver for the oracle under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Runs every oracle function on small random inputs (odd sizes, full range and random
 * bands, both transition modes, every number of paths, the layered merge with and
 * without its occlusion weight) so that the sanitizers see each code path; also checks
 * that the fast transition equals the definition (Section 3.3) on every input. Exit status 0 on success. Built and run by tests/test_oracle_sanitize.py;
 * test infrastructure only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_downsample(const uint8_t *in, int W, int H, uint8_t *out);
void orc_census5x5(const uint8_t *img, int W, int H, uint32_t *out);
void orc_cost(const uint32_t *cl, const uint32_t *cr, int W, int H, const int16_t *lo,
              const uint8_t *len, int cap, uint8_t *cost);
int orc_aggregate(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                  int cap, int num_paths, uint32_t path_mask, int lambda, int tau, int mode,
                  int64_t *S, int64_t *Lscratch, int64_t *per_path);
void orc_wta_lr(const int64_t *S, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                int cap, int lr_max_diff, int16_t *dl_out, int16_t *dr_out, int16_t *out);
int orc_propagate(const int16_t *dl_coarse, int Wc, int Hc, int W, int H, int Dl, int R,
                  int16_t *lo);
int orc_layered(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                int cap, int num_layers, int lambda, int tau, int occ, int mode, int64_t *M,
                int64_t *per_layer);
int orc_aggregate_g(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                    int cap, int num_paths, uint32_t path_mask, int lambda, int tau,
                    const uint8_t *img, int sigma, int mode, int64_t *S, int64_t *Lscratch,
                    int64_t *per_path);
int orc_layered_g(const uint8_t *cost, int W, int H, int D, const int16_t *lo, const uint8_t *len,
                  int cap, int num_layers, int lambda, int tau, int occ, const uint8_t *img,
                  int sigma, int mode, int64_t *M, int64_t *per_layer);

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint32_t next(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (uint32_t)rng;
}

static int run(int W, int H, int D, int banded, int paths, int tau) {
    const long n = (long)W * H;
    uint8_t *L = malloc(n), *R = malloc(n);
    for (long i = 0; i < n; ++i) {
        L[i] = (uint8_t)(next() % 256);
        R[i] = (uint8_t)(next() % 256);
    }
    uint8_t *half = malloc((size_t)(W / 2 > 0 ? W / 2 : 1) * (H / 2 > 0 ? H / 2 : 1));
    if (W >= 2 && H >= 2) orc_downsample(L, W, H, half);
    uint32_t *cl = malloc(sizeof(uint32_t) * n), *cr = malloc(sizeof(uint32_t) * n);
    orc_census5x5(L, W, H, cl);
    orc_census5x5(R, W, H, cr);
    int cap = D;
    int16_t *lo = NULL;
    uint8_t *len = NULL;
    if (banded) {
        cap = D < 5 ? D : 5;
        lo = malloc(sizeof(int16_t) * n);
        len = malloc(n);
        for (long i = 0; i < n; ++i) {
            len[i] = (uint8_t)(1 + next() % cap);
            lo[i] = (int16_t)(next() % (D - len[i] + 1));
        }
    }
    uint8_t *cost = malloc((size_t)n * cap);
    orc_cost(cl, cr, W, H, lo, len, cap, cost);
    int64_t *S0 = malloc(sizeof(int64_t) * n * cap), *S1 = malloc(sizeof(int64_t) * n * cap);
    int64_t *scr = malloc(sizeof(int64_t) * n * cap);
    int64_t *per = malloc(sizeof(int64_t) * n * cap * 8);
    int bad = 0;
    if (orc_aggregate(cost, W, H, D, lo, len, cap, paths, 0, 8, tau, 0, S0, scr, per)) bad = 1;
    if (orc_aggregate(cost, W, H, D, lo, len, cap, paths, 0, 8, tau, 1, S1, scr, NULL)) bad = 1;
    for (long i = 0; i < n * cap; ++i)
        if (S0[i] != S1[i]) {
            bad = 1;
            break;
        }
    /* layered merge: both transition modes agree, with and without the occlusion weight */
    for (int occ = 0; occ < 2; ++occ) {
        if (orc_layered(cost, W, H, D, lo, len, cap, 4, 8, tau, occ, 0, S0, per)) bad = 1;
        if (orc_layered(cost, W, H, D, lo, len, cap, 4, 8, tau, occ, 1, S1, NULL)) bad = 1;
        for (long i = 0; i < n * cap; ++i)
            if (S0[i] != S1[i]) {
                bad = 1;
                break;
            }
    }
    /* gradient-weighted transition (left image as the weight source), both modes agree */
    if (orc_aggregate_g(cost, W, H, D, lo, len, cap, paths, 0, 8, tau, L, 5, 0, S0, scr, per)) bad = 1;
    if (orc_aggregate_g(cost, W, H, D, lo, len, cap, paths, 0, 8, tau, L, 5, 1, S1, scr, NULL)) bad = 1;
    for (long i = 0; i < n * cap; ++i)
        if (S0[i] != S1[i]) {
            bad = 1;
            break;
        }
    if (orc_layered_g(cost, W, H, D, lo, len, cap, 4, 8, tau, 1, L, 5, 0, S0, per)) bad = 1;
    if (orc_layered_g(cost, W, H, D, lo, len, cap, 4, 8, tau, 1, L, 5, 1, S1, NULL)) bad = 1;
    for (long i = 0; i < n * cap; ++i)
        if (S0[i] != S1[i]) {
            bad = 1;
            break;
        }
    int16_t *dl = malloc(sizeof(int16_t) * n), *dr = malloc(sizeof(int16_t) * n);
    int16_t *out = malloc(sizeof(int16_t) * n);
    orc_wta_lr(S1, W, H, D, lo, len, cap, 1, dl, dr, out);
    const int W2 = 2 * W + 1, H2 = 2 * H + 1, D2 = 2 * D;
    int16_t *lo2 = malloc(sizeof(int16_t) * W2 * H2);
    orc_propagate(dl, W, H, W2, H2, D2, 4, lo2);
    free(L); free(R); free(half); free(cl); free(cr); free(lo); free(len); free(cost);
    free(S0); free(S1); free(scr); free(per); free(dl); free(dr); free(out); free(lo2);
    return bad;
}

int main(void) {
    const int shapes[][3] = {{1, 1, 1}, {5, 3, 3}, {7, 5, 4}, {16, 9, 8}, {33, 17, 12}, {3, 40, 6}};
    int fails = 0;
    for (unsigned s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s)
        for (int banded = 0; banded < 2; ++banded)
            for (int paths = 1; paths <= 8; paths *= 2)
                for (int tau = 1; tau <= 5; tau += 2) {
                    const int r = run(shapes[s][0], shapes[s][1], shapes[s][2], banded, paths, tau);
                    if (r) {
                        printf("mismatch: W=%d H=%d D=%d banded=%d paths=%d tau=%d\n", shapes[s][0],
                               shapes[s][1], shapes[s][2], banded, paths, tau);
                        ++fails;
                    }
                }
    printf("%s\n", fails ? "FAIL" : "ok");
    return fails ? 1 : 0;
}
