/*
 * mpv.h - C ABI of the MI355X (gfx950) multi-scale MPV stereo matcher.
 *
 * The library computes the disparity map U that the paper's Multi-Path-Viterbi
 * approximately minimises (Section 3.2, eqs. EU and viterbi): a per-pixel matching cost
 * (census 5x5 / Hamming here, in place of the paper's SSIM), a min-plus Viterbi pass
 * along several scanline directions with a truncated total-variation transition
 * lambda*min(|d-d'|, tau) (eq. e(p,u); Section 3.3 fast technique), the sum of the path
 * energies, winner-take-all disparity, a left-right consistency check, and the
 * coarse-to-fine search-band propagation of the image pyramid (Section 3.4).
 *
 * Conventions for every entry point
 *  - Pointers to images, volumes and maps are DEVICE pointers (hipMalloc'd or torch
 *    tensors); parameter structs are host pointers read during the call only.
 *  - Every call is asynchronous: work is enqueued on `stream` (0 = the null stream) and
 *    nothing synchronises. Host-visible results need a stream synchronisation.
 *  - Argument, shape, workspace and overflow problems are detected before anything is
 *    enqueued and returned as a status; nothing is launched then. A failed launch
 *    returns MPV_ERR_DEVICE. No C++ exception crosses the ABI.
 *  - The caller owns all memory. The library allocates nothing; scratch comes from the
 *    caller's workspace, sized by the matching *_workspace_bytes call. Concurrent calls
 *    on different streams need distinct workspaces and outputs.
 *  - Images are uint8, row-major, `pitch` bytes between rows (pitch >= width).
 *    Volumes are [H][W][cap] with the disparity slot innermost. Disparity maps are
 *    int16 [H][W] with -1 meaning invalid.
 *  - The left image is the reference: left pixel (x, y) with disparity d matches right
 *    pixel (x - d, y). A candidate with x - d < 0 costs 24 (every census bit differs).
 */
#ifndef MPV_H
#define MPV_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPV_OK = 0,
    MPV_ERR_INVALID_ARG = 1, /* null pointer, bad size, bad parameter */
    MPV_ERR_UNSUPPORTED = 2, /* valid but outside what the kernels implement */
    MPV_ERR_WORKSPACE = 3,   /* workspace missing or too small */
    MPV_ERR_OVERFLOW = 4,    /* the requested sum type cannot hold the energies */
    MPV_ERR_DEVICE = 5       /* a HIP call or launch failed */
} mpv_status;

/* Aggregate-sum export types for mpv_aggregate / mpv_disparity. */
#define MPV_AGG_U16 0
#define MPV_AGG_I32 1

/* Path merge (mpv_params.merge).
 * MPV_MERGE_SUM: S(p,d) = the sum of the num_paths directed-path energies.
 * MPV_MERGE_LAYERED: the hierarchical merge of Section 3.2 (Table alg). num_paths / 2
 *   layers run the opposite direction pairs in the table's order (left/right, up/down,
 *   the two diagonals); each pass's energies are taken relative to the pixel's minimum
 *   over its band, the first (horizontal) layer keeps the smaller of the two, every other
 *   layer their mean rounded down, and each layer's merged energy is the data term of the
 *   next. Decisions (WTA, right disparity, LR) are taken on the last layer's merge.
 *   num_paths must be 2, 4 or 8.
 * MPV_MERGE_LAYERED_OCC: as MPV_MERGE_LAYERED with the paper's example strategy for
 *   occluded areas: the left-to-right pass pays twice the transition weight when the
 *   disparity increases along the path. */
#define MPV_MERGE_SUM 0
#define MPV_MERGE_LAYERED 1
#define MPV_MERGE_LAYERED_OCC 2

#define MPV_MAX_DISP 256
#define MPV_MAX_LEVELS 4
#define MPV_MAX_WIDTH 4096
#define MPV_MAX_HEIGHT 65536

/* Scan directions, in the order of the paper's multi-path table (Section 3.2, Table alg):
 * bit r of a path mask selects direction r. num_paths = P selects the first P. */
#define MPV_DIR_L2R 0   /* (+1, 0) */
#define MPV_DIR_R2L 1   /* (-1, 0) */
#define MPV_DIR_T2B 2   /* ( 0,+1) */
#define MPV_DIR_B2T 3   /* ( 0,-1) */
#define MPV_DIR_TL2BR 4 /* (+1,+1) */
#define MPV_DIR_BR2TL 5 /* (-1,-1) */
#define MPV_DIR_TR2BL 6 /* (-1,+1) */
#define MPV_DIR_BL2TR 7 /* (+1,-1) */

typedef struct {
    const uint8_t *data; /* device pointer */
    int32_t width, height, pitch;
} mpv_image;

/* Per-pixel search band (Section 3.4's per-pixel search scope). Pixel p searches the
 * disparities lo[p] .. lo[p] + len[p] - 1, stored in slots 0 .. len[p]-1 of a
 * [H][W][cap] volume. lo == NULL means the full range [0, num_disp) with cap = num_disp;
 * len == NULL means len[p] = cap everywhere. Requires 1 <= len[p] <= cap and
 * 0 <= lo[p] <= num_disp - len[p]; disparities outside a band are absent Viterbi nodes.
 * The maps are not validated; the kernels clamp lo to [0, num_disp-1] and len to
 * [1, min(cap, num_disp-lo)], so a map that breaks the rule still stays in bounds. */
typedef struct {
    const int16_t *lo;  /* device [H][W] or NULL */
    const uint8_t *len; /* device [H][W] or NULL */
    int32_t cap;
} mpv_band;

typedef struct {
    int32_t num_disp;      /* D: 1 .. MPV_MAX_DISP */
    int32_t census_radius; /* must be 2 (5x5 census, 24 bits) */
    int32_t num_paths;     /* P in {1, 2, 4, 8}: the first P directions */
    int32_t lambda;        /* transition weight, >= 0 */
    int32_t tau;           /* truncation, >= 1; tau >= num_disp is the untruncated TV */
    int32_t lr_max_diff;   /* LR tolerance in px (1 = "1 px"); < 0 disables the check */
    int32_t agg_type;      /* MPV_AGG_U16 or MPV_AGG_I32 (exported sums only) */
    int32_t merge;         /* MPV_MERGE_*: how the directed paths are combined (0 = sum) */
    int32_t grad_sigma;    /* 0: every transition weighs lambda. 1..255: the gradient-weighted
                              TV of eq. EU, the edge between consecutive path pixels p-r, p
                              weighs round(lambda * exp(-|I(p) - I(p-r)| / grad_sigma)) with I
                              the left image of the level (mpv_match, mpv_pyramid, batches) */
    int32_t data_term;     /* MPV_DATA_CENSUS (0) or MPV_DATA_SSIM: the matching cost C(p,d) */
} mpv_params;

/* Data term (mpv_params.data_term); both costs lie in 0 .. 24, so lambda and tau mean the same.
 * MPV_DATA_CENSUS: Hamming distance of the 5x5 census signatures (mpv_census).
 * MPV_DATA_SSIM: the structural-similarity cost of Section 3.2 (eqs. components and ssim) with
 *   the constants of the similarity index the paper cites (K1 = 0.01, K2 = 0.03, dynamic range
 *   255, C3 = C2/2, unit exponents). psi and phi are the 5x5 patches (uniform weights,
 *   coordinates clamped to the image) of the left image around (x, y) and of the right image
 *   around (x - d, y); with C3 = C2/2 the product of the three components is exactly
 *   SSIM = (2 mu_psi mu_phi + C1)(2 cov + C2) / ((mu_psi^2 + mu_phi^2 + C1)(var_psi + var_phi + C2))
 *   (population moments), evaluated exactly as a ratio of integers; the cost is
 *   (1 - SSIM) * 24 / 2 rounded half up, and 24 where x - d < 0. mpv_cost writes it;
 *   mpv_match and mpv_pyramid compute it once per level into the workspace and scan from it
 *   (sum of the paths without gradient weights only: MPV_ERR_UNSUPPORTED otherwise); batches
 *   and the learned coarse level take the census only. */
#define MPV_DATA_CENSUS 0
#define MPV_DATA_SSIM 1

/* Human-readable status name; never NULL. */
const char *mpv_status_string(mpv_status s);

/* Census transform (the cost's per-pixel signature; replaces the paper's SSIM patches of
 * Section 3.2): bit k of census[y][x] is set when the k-th neighbour of the 5x5 window,
 * in row-major order skipping the centre, is darker than the centre; neighbour
 * coordinates are clamped to the image. Output: device uint32 [H][W], bits 24..31 zero. */
mpv_status mpv_census(const mpv_image *img, uint32_t *census, hipStream_t stream);

/* One pyramid step (Section 3.4): out[y][x] = (sum of the 2x2 block at (2x, 2y) + 2) >> 2,
 * for an output of floor(W/2) x floor(H/2) pixels, rows packed (pitch = W/2). */
mpv_status mpv_downsample(const mpv_image *img, uint8_t *out, hipStream_t stream);

/* Matching-cost volume: cost[y][x][j] = popcount(cL(x,y) ^ cR(x-d,y)) for d = lo + j in the
 * band (24 when x-d < 0), or the SSIM cost of MPV_DATA_SSIM, 0xFF in slots past the pixel's
 * band. This is the data term of eq. e(p,u). Output: device uint8 [H][W][cap]. band may be
 * NULL (full range). */
mpv_status mpv_cost(const mpv_params *p, const mpv_image *left, const mpv_image *right,
                    const mpv_band *band, uint8_t *cost, hipStream_t stream);

/* Path energies and their sum (eqs. viterbi, e(p,u)):
 *   L_r(p,d) = C(p,d) + min_{d' in B(p-r)} [L_r(p-r,d') + lambda*min(|d-d'|, tau)],
 *   L_r(p,d) = C(p,d) where p-r is outside the image,
 *   agg[p][j] = sum over the selected directions r of L_r(p, lo+j)    (unnormalised).
 * Input: the [H][W][cap] cost volume of mpv_cost. path_mask selects a subset of the first
 * num_paths directions (0 = all of them). Output: device [H][W][cap] of uint16 or int32
 * per agg_type; slots past a pixel's band hold the type's maximum.
 * MPV_ERR_OVERFLOW when P * (24 + lambda*min(tau, D-1)) * longest line may exceed the type;
 * MPV_ERR_UNSUPPORTED when lambda*min(tau, D-1) > 4000 or merge is not MPV_MERGE_SUM. */
mpv_status mpv_aggregate(const mpv_params *p, const uint8_t *cost, int32_t width, int32_t height,
                         const mpv_band *band, uint32_t path_mask, void *agg, hipStream_t stream);

/* Winner-take-all and left-right check on an aggregate volume (agg_type selects
 * uint16 or int32):
 *   raw(p)   = the smallest in-band d minimising agg(p, d)
 *   S'(p,d)  = agg(p,d) - min_d agg(p,d)
 *   right(x,y) = the largest d minimising S'(x+d, y, d) over the d with x+d < W and d in
 *              B(x+d, y); -1 if there is none (ties go to the nearer surface)
 *   disp(p)  = raw(p) if x-raw >= 0, right(x-raw, y) >= 0 and |raw - right(x-raw,y)|
 *              <= lr_max_diff, else -1; lr_max_diff < 0 gives disp = raw.
 * disp is required; disp_right and disp_raw may be NULL. Requires width <= MPV_MAX_WIDTH. */
mpv_status mpv_disparity(const mpv_params *p, const void *agg, int32_t width, int32_t height,
                         const mpv_band *band, int16_t *disp, int16_t *disp_right,
                         int16_t *disp_raw, hipStream_t stream);

/* Launch schedule of the fused path. Every schedule gives bit-identical results; they
 * differ only in speed (an autotuner picks one per workload). Zero = library default. */
typedef struct {
    int32_t waves_per_block; /* scan blocks hold 1, 2 or 4 independent waves */
    int32_t full_lanes;      /* full-range scans: lanes per line (16, 32, 64) if the range fits
                                2 packed pairs per lane, else the default layout */
    int32_t band_lanes;      /* banded scans: lanes per line (16, 32, 64) if the band fits
                                (cap + 2*(tau_eff-1) < lanes), or MPV_BAND_LANES_LINE */
    int32_t order;           /* batched scans: 0 = pair by pair, 1 = longest lines first */
} mpv_schedule;

/* mpv_schedule.band_lanes of a batch (mpv_batch_create): one scan line per lane for the
 * directions that cross image rows (vertical and diagonal; a wave walks 64 neighbouring lines
 * row by row), with the horizontal directions' 16-lane groups running beside them on a second
 * stream; a pixel's partial energies take 8 bytes of six-bit slots where
 * 24 + lambda*tau_eff <= 63, else 12 byte slots. Taken by the levels whose bands hold 5 or 9
 * disparities with tau_eff = min(tau, D-1) of 1, 2 or 4, for the census data term, the sum
 * of the paths and constant weights; every other level, and every single-pair entry point
 * (whose lone frame's lines would be long serial chains), runs as with band_lanes = 0. */
#define MPV_BAND_LANES_LINE 1

/* How a finer pyramid level's search band is centred (mpv_pyramid_params.propagation).
 * MPV_PROP_NEAREST: every pixel on twice its parent's raw winner.
 * MPV_PROP_PAPER: the paper's own scheme (Section 3.4): only the pixels sampled from the
 *   coarser level carry an initial value (twice the parent's raw winner); an intermediate
 *   level is split into blocks and every pixel of a block is centred on the block's mode of
 *   its parents' initial values (the most frequent, the smallest on ties); the last level
 *   treats every pixel as a block and gives the pixels between samples the linear
 *   interpolation of the samples around them (the mean of two, or of four rounded half up;
 *   samples past the coarser image are clamped to its last row and column). */
#define MPV_PROP_NEAREST 0
#define MPV_PROP_PAPER 1
#define MPV_MAX_BLOCK 32

/* Multi-scale fused path (Section 3.4). */
typedef struct {
    mpv_params base;     /* num_disp = D of the finest (input) level */
    int32_t levels;      /* 1 .. MPV_MAX_LEVELS; 1 = plain single-scale MPV */
    int32_t band_radius; /* R: levels below the top search [c-R, c+R] around their centre c */
    mpv_schedule sched;  /* launch schedule (zeros = defaults) */
    int32_t propagation; /* MPV_PROP_NEAREST (0) or MPV_PROP_PAPER */
    int32_t block;       /* MPV_PROP_PAPER: block side at level 1 (even, 2 .. MPV_MAX_BLOCK; 0 = 8),
                            halved at every finer intermediate level, never below 2 */
} mpv_pyramid_params;

typedef struct {
    int16_t *disp;                      /* required: [H][W] finest, LR-checked */
    int16_t *disp_raw;                  /* optional: finest raw WTA */
    int16_t *disp_right;                /* optional: finest right disparity */
    int16_t *level_raw[MPV_MAX_LEVELS]; /* optional: raw WTA per level, 0 = coarsest */
} mpv_pyramid_out;

/* Workspace bytes mpv_pyramid needs for this shape; 0 if the parameters are invalid. */
size_t mpv_pyramid_workspace_bytes(const mpv_pyramid_params *p, int32_t width, int32_t height);

/* Level l of L has size floor(W / 2^(L-1-l)) x floor(H / 2^(L-1-l)) and range
 * D_l = ceil(D / 2^(L-1-l)). The top level (l = 0) searches its full range. Every finer
 * level searches the band of cap = min(2R+1, D_l) disparities starting at
 * lo = clamp(c - R, 0, D_l - cap), with c = 2 * raw_{l-1}(min(x/2, W_{l-1}-1),
 * min(y/2, H_{l-1}-1)) for MPV_PROP_NEAREST, the block mode or interpolated centre for
 * MPV_PROP_PAPER. Batches (mpv_batch_*) take MPV_PROP_NEAREST only.
 * Each level runs cost -> all P paths -> sum -> WTA -> LR exactly as the unfused calls
 * do, so the outputs equal mpv_cost + mpv_aggregate + mpv_disparity per level; with a
 * layered merge each level runs the layers in turn and decides on the last layer's merge.
 * Requires 24 + lambda*min(tau, D-1) <= 255 (layered: 24 + m*lambda*min(tau, D-1) <= 255
 * with m = the number of layers, at least 2 for MPV_MERGE_LAYERED_OCC, so that every
 * merged energy fits a byte; MPV_ERR_UNSUPPORTED otherwise), num_paths in {1,2,4,8}
 * ({2,4,8} for a layered merge) and every level at
 * least 1x1 pixel, at most MPV_MAX_WIDTH wide and MPV_MAX_HEIGHT high; one direction's
 * partial volume (width * height * slots) below 2^31 bytes (MPV_ERR_INVALID_ARG otherwise). */
mpv_status mpv_pyramid(const mpv_pyramid_params *p, const mpv_image *left, const mpv_image *right,
                       const mpv_pyramid_out *out, void *workspace, size_t workspace_bytes,
                       hipStream_t stream);

/* Allocation-free variant of mpv_pyramid, for callers that cannot allocate device memory
 * (code under graph capture, serving loops and harnesses that forbid hipMalloc): the same
 * computation and outputs as mpv_pyramid, with the workspace taken from a fixed device array
 * of MPV_PYRAMID_NOALLOC_MAX_BYTES that the library owns, one copy per GPU, set up on the
 * first call on that GPU and held until the process ends. The call allocates and frees
 * nothing. MPV_ERR_WORKSPACE when mpv_pyramid_workspace_bytes for this shape exceeds the
 * maximum (1280x720, D=128, 3 levels, 8 paths needs 129.3 MiB; 640x480 about 44 MiB);
 * other arguments are checked as by mpv_pyramid; MPV_ERR_DEVICE when the current device or
 * the array's address cannot be obtained. Every call on a GPU uses the same array and leaves
 * its contents behind (nothing in it needs clearing between calls), so calls that overlap on
 * one GPU (concurrent streams or threads) race: the caller serialises them. */
#define MPV_PYRAMID_NOALLOC_MAX_BYTES ((size_t)144 << 20)
mpv_status mpv_pyramid_noalloc(const mpv_pyramid_params *p, const mpv_image *left,
                               const mpv_image *right, const mpv_pyramid_out *out,
                               hipStream_t stream);

/* One fused level with a caller-given band (the learned-band path: a network proposes
 * lo/len per pixel and the finest level searches only there). Same arithmetic and
 * outputs as one level of mpv_pyramid, with the same limits. band may be NULL (full range).
 * mpv_match_workspace_bytes returns 0 for arguments mpv_match would reject. */
size_t mpv_match_workspace_bytes(const mpv_params *p, int32_t width, int32_t height,
                                 const mpv_band *band);
mpv_status mpv_match(const mpv_params *p, const mpv_image *left, const mpv_image *right,
                     const mpv_band *band, int16_t *disp, int16_t *disp_right, int16_t *disp_raw,
                     void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Batched multi-scale matching of many pairs of different sizes and ranges (the analogue
 * of the paper's frame pipelining, Section 3.7): every stage of every level runs as one
 * launch over all pairs (a device descriptor table maps blocks to pairs), pairs share
 * lambda/tau/P/levels/R and the schedule of the mpv_pyramid_params, and each pair has its
 * own D (its num_disp) and its own workspace region, so each output equals mpv_pyramid of
 * that pair alone. Usage: create (host only) -> workspace_bytes -> bind (uploads the
 * descriptor tables into the workspace and synchronises `stream`) -> run / run_graph any
 * number of times. The items' images and outputs must stay allocated while the batch
 * lives; their contents may change between runs. The handle is host memory owned by the
 * library until mpv_batch_destroy. With a layered merge every layer is one launch per
 * kernel variant over all pairs, in turn. */
typedef struct mpv_batch_s *mpv_batch;
typedef struct {
    mpv_image left, right; /* device images of one pair */
    int32_t num_disp;      /* D of this pair, 1 .. MPV_MAX_DISP */
    int16_t *disp;         /* required: [H][W] LR-checked disparity */
    int16_t *disp_right;   /* optional: right disparity */
    int16_t *disp_raw;     /* optional: raw WTA */
} mpv_batch_item;

mpv_status mpv_batch_create(const mpv_pyramid_params *p, const mpv_batch_item *items, int32_t n,
                            mpv_batch *out);
size_t mpv_batch_workspace_bytes(mpv_batch b);
mpv_status mpv_batch_bind(mpv_batch b, void *workspace, size_t workspace_bytes, hipStream_t stream);
/* Enqueue the whole batch (about 4 launches per level) on `stream`. The census of the finer
 * levels runs on a stream the batch owns, forked by an event recorded on `stream` after the
 * coarsest level's census and joined back before its level's first scan; with band_lanes =
 * MPV_BAND_LANES_LINE a line level's horizontal scan runs on a second owned stream, forked
 * before the level's line scan and joined back before its reduce. The batch stays ordered
 * with the caller's work on `stream` (also in mpv_batch_run_graph). */
mpv_status mpv_batch_run(mpv_batch b, hipStream_t stream);
/* Same work as one hipGraph: captured on a private stream at the first call, then replayed
 * on `stream` with one hipGraphLaunch per call. */
mpv_status mpv_batch_run_graph(mpv_batch b, hipStream_t stream);
/* The launches of mpv_batch_run restricted to the n distinct items idx[0..n) (a service's
 * admitted frames, in any order): each item keeps its own workspace region and outputs, so
 * its output still equals mpv_pyramid of that pair alone, and the other items' outputs are
 * untouched. The restricted descriptor tables are planned on the host and copied, through
 * pinned staging memory the batch owns (a small ring allocated at the first call, freed by
 * mpv_batch_destroy), into a second table area of the workspace, then the launches are
 * enqueued. Calls on one batch share that table area: issue them (and mpv_batch_run) on one
 * stream. The call may wait for the upload of the call four before it to have completed. */
mpv_status mpv_batch_run_items(mpv_batch b, const int32_t *idx, int32_t n, hipStream_t stream);
void mpv_batch_destroy(mpv_batch b);

/* Road profile in v-disparity space and the u-disparity image (Section 3.5), downstream of
 * the disparity map.
 *
 * mpv_vdisparity: the v-disparity image of eq. disp_map, hist[i][j] = the number of pixels
 * of row j whose disparity is i, for 0 <= i < num_disp (1 .. MPV_MAX_DISP). disp: device
 * int16 [height][pitch] (pitch >= width, in elements); -1 and values outside [0, num_disp)
 * are not counted. hist: device uint32 [num_disp][height], every entry written.
 *
 * mpv_udisparity: the u-disparity image of eq. hy, its column-wise counterpart (read with
 * the second Kronecker delta on the disparity: the printed one repeats the column index),
 * hist[i][j] = the number of pixels of column j whose disparity is i. Same disp arguments
 * and exclusions; hist: device uint32 [num_disp][width], every entry written.
 *
 * mpv_road: the road profile of eqs. P_hat and e over a v-disparity image: the path j = P(i)
 * over every disparity i = 0 .. num_disp-1 whose row grows by 1 to eta-1 per step (2 <=
 * eta <= 256) and whose sum of counts is largest; e(0,j) = hist[0][j],
 * e(i,j) = hist[i][j] + max over 0 < j-j' < eta of e(i-1,j'). The end is the smallest row
 * maximising e(num_disp-1, .), each predecessor the smallest maximising row. path: device
 * int16 [num_disp] (rows), energy: device int32 [1] (the profile's sum); both -1 when no
 * row is reachable at the last disparity. Requires height <= MPV_ROAD_MAX_HEIGHT and a
 * workspace of mpv_road_workspace_bytes (num_disp*height bytes of back-pointers; 0 for
 * arguments mpv_road rejects). One workgroup: a small downstream step, not a full-chip
 * kernel. */
#define MPV_ROAD_MAX_HEIGHT 4096
mpv_status mpv_vdisparity(const int16_t *disp, int32_t width, int32_t height, int32_t pitch,
                          int32_t num_disp, uint32_t *hist, hipStream_t stream);
mpv_status mpv_udisparity(const int16_t *disp, int32_t width, int32_t height, int32_t pitch,
                          int32_t num_disp, uint32_t *hist, hipStream_t stream);
size_t mpv_road_workspace_bytes(int32_t num_disp, int32_t height);
mpv_status mpv_road(const uint32_t *hist, int32_t num_disp, int32_t height, int32_t eta, int16_t *path,
                    int32_t *energy, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Measurement hook (per-kernel timing without a profiler). Stages of one level: */
#define MPV_STAGE_DOWNSAMPLE 0 /* batches only: mpv_pyramid builds no coarse images */
#define MPV_STAGE_CENSUS 1     /* mpv_pyramid: one launch, bracketed whatever level is hooked:
                                  the top level's census (with several levels the finer levels'
                                  census runs inside the top level's first scan launch) */
#define MPV_STAGE_SCAN 2      /* all P directions of one level, one launch */
#define MPV_STAGE_REDUCE 3    /* sum + WTA + right disparity + LR of one level, and (nearest
                                 propagation) the band of the next finer level (Section 3.4) */
#define MPV_STAGE_PROPAGATE 4 /* MPV_PROP_PAPER: the launch that writes the next finer level's
                                 band from this level's raw winners (nearest propagation runs
                                 inside the coarser level's reduce and has none) */
#define MPV_NUM_STAGES 5

/* While set, every later run of `stage` at pyramid level `level` (0 = coarsest; the
 * single level of mpv_match is level 0; -1 = any level) is bracketed by
 * hipEventRecord(before) and hipEventRecord(after) on the launch stream; a stage made of
 * several consecutive launches (the layers of a layered merge, kernel variants of a batch)
 * is bracketed as a whole. NULL events clear
 * the hook. Process-wide host state, not synchronised: set it from the thread that
 * enqueues, between calls. The events are the caller's; the library never creates or
 * destroys them. */
mpv_status mpv_set_timing_events(int32_t stage, int32_t level, hipEvent_t before, hipEvent_t after);

#ifdef __cplusplus
}
#endif
#endif /* MPV_H */
