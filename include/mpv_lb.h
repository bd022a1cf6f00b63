/*
 * mpv_lb.h - C ABI of the learned band proposal (a small convolutional network, BF16
 * operands with FP32 accumulation on MFMA) that predicts, from the coarsest pyramid level,
 * the disparity band each finest-level pixel searches. This replaces the propagated
 * per-pixel search scopes of the paper's multi-scale scheme (Section 3.4) by learned ones;
 * the finest level then runs mpv_match with the predicted band.
 *
 * Conventions are those of mpv.h (device pointers, caller-owned memory, asynchronous on
 * `stream`, synchronous argument errors). Activations are NHWC: n images of h x w pixels,
 * channel innermost, bf16 stored as uint16_t bit patterns. A layer's FP32 master weights
 * are w[3][3][cin][cout] (tap (ky, kx) reads input pixel (y+ky-1, x+kx-1), zero padding)
 * and b[cout]. All reductions run in a fixed order: results do not depend on scheduling.
 */
#ifndef MPV_LB_H
#define MPV_LB_H

#include "mpv.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MPV_LB_FEATURES 8

/* Coarse level and features. Runs the fused single-level MPV (full range, P paths, LR
 * check) on the coarse pair, then writes 8 features per coarse pixel:
 *   0: I/255   1: raw/D   2: [LR-valid]   3..6: S'(raw-1), S'(raw+1), S'(raw-2), S'(raw+2)
 *   (disparities clamped to [0, D-1])   7: min over |d-raw| > 1 of S' (1 if none),
 * with S' = the sum of path energies minus its per-pixel minimum, channels 3..7 divided by
 * P * (24 + lambda*min(tau, D-1)); values rounded to bf16 (nearest, ties to even).
 * feat: bf16 [H0][W0][8]; raw0, disp0: int16 [H0][W0] (raw WTA, LR-checked).
 * The features are defined on the sum of the paths: a layered merge is MPV_ERR_UNSUPPORTED
 * (workspace size 0). */
size_t mpv_lb_coarse_workspace_bytes(const mpv_params *p, int32_t W0, int32_t H0);
mpv_status mpv_lb_coarse(const mpv_params *p, const mpv_image *left0, const mpv_image *right0,
                         uint16_t *feat, int16_t *raw0, int16_t *disp0, void *workspace,
                         size_t workspace_bytes, hipStream_t stream);

/* Packed bf16 weights of one layer (cin, cout multiples of 4 up to 32, or cout = 3):
 * forward: [round16(cout)][round32(9*cin)], k = (ky*3+kx)*cin + ci;
 * backward-data: [round16(cin)][round32(9*round4(cout))], taps mirrored, k = tap*round4(cout) + co
 * (the reduction padded to the 32-deep steps of the bf16 MFMA). */
size_t mpv_lb_packed_elems(int32_t cin, int32_t cout);
size_t mpv_lb_packed_bwd_elems(int32_t cin, int32_t cout);
mpv_status mpv_lb_pack(const float *w, int32_t cin, int32_t cout, uint16_t *wfwd, uint16_t *wbwd,
                       hipStream_t stream);

/* y = conv3x3(x, w) + bias (bias may be NULL), then ReLU if relu, then multiplied by
 * [mask > 0] if mask (bf16, `mask_stride` channels per pixel) is given. x has cin channels
 * (4, 8 or 32). y has y_stride >= cout channels per pixel (channels cout..y_stride-1 are
 * written as 0) and is fp32 when y_f32, bf16 otherwise. `w` is the forward packing (or the
 * backward-data packing with cin and cout exchanged, which computes dL/dx from dL/dy). */
mpv_status mpv_lb_conv(const uint16_t *x, int32_t n, int32_t h, int32_t w, int32_t cin,
                       const uint16_t *wpacked, const float *bias, int32_t cout, int32_t relu,
                       const uint16_t *mask, int32_t mask_stride, void *y, int32_t y_stride,
                       int32_t y_f32, hipStream_t stream);

/* Weight and bias gradients of a layer: dw[3][3][cin][cout] = sum over pixels of
 * x(shifted by the tap) * dz, db[cout] = sum of dz; dz has dz_stride channels per pixel.
 * Split over pixel chunks with a fixed-order final sum. */
size_t mpv_lb_dw_workspace_bytes(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout);
mpv_status mpv_lb_conv_dw(const uint16_t *x, const uint16_t *dz, int32_t dz_stride, int32_t n,
                          int32_t h, int32_t w, int32_t cin, int32_t cout, float *dw, float *db,
                          void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Heads and loss of the network output o (fp32, 4 per coarse pixel, channel 3 unused):
 *   center = 4*raw0 + o0, width = 2 + clamp(o1, 0, 14), conf = clamp(o2, 0, 1);
 * per labelled fine pixel q of the coarse pixel's 4x4 block (labels: int16 [n][H][W],
 * -1 = none): smoothL1(center - d*) + max(0, 2|d* - center| + 2 - width) + beta*width +
 * (conf - [|d* - center| <= width/2])^2, times inv_count. Writes dL/do as bf16
 * [n][hc][wc][4] and one loss partial per 256 coarse pixels (fixed-order sums). */
mpv_status mpv_lb_loss(const float *o, const int16_t *raw0, const int16_t *labels, int32_t n,
                       int32_t hc, int32_t wc, int32_t H, int32_t W, float beta, float inv_count,
                       uint16_t *dz, float *loss_partials, hipStream_t stream);

/* Adam on FP32 masters (bias-corrected, step >= 1). */
mpv_status mpv_lb_adam(float *p, float *m, float *v, const float *g, int64_t count, float lr,
                       float beta1, float beta2, float eps, int32_t step, hipStream_t stream);

/* Fine-level bands from the network output of one image: center rounded half up, width
 * 2 + clamp(round half up(o1), 0, 14); a coarse pixel with conf < theta gets width 16.
 * Every fine pixel (x, y) takes coarse pixel (min(x/4, wc-1), min(y/4, hc-1)):
 * len = min(width, D), lo = clamp(center - len/2, 0, D - len). *n_low (device int32,
 * zeroed by the call) receives the number of low-confidence coarse pixels. */
mpv_status mpv_lb_bands(const float *o, const int16_t *raw0, int32_t wc, int32_t hc, int32_t W,
                        int32_t H, int32_t D, float theta, int16_t *lo, uint8_t *len,
                        int32_t *n_low, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* MPV_LB_H */
