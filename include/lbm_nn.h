/*
 * lbm_nn.h -- C ABI of the warm-start network kernels (part of liblbm.so).
 *
 * The network predicts near-steady fields (u, v, T, phi) of a channel from
 * its wall-heating law and properties; the LBM then starts from them
 * (lbm_init_device) instead of from rest.  The network is a small U-Net of
 * 3x3 convolutions; these entry points are its building blocks: forward and
 * both backward passes of the convolution on BF16 matrix cores with FP32
 * accumulation, the elementwise pieces, the loss, Adam, and the conversions
 * between LBM channels and network tensors.
 *
 * Conventions:
 *   - tensors are device memory, NHWC (channels fastest), x periodic and
 *     zero padding in y (the channel's walls); "bf16" buffers hold bfloat16
 *     bit patterns in uint16_t;
 *   - convolution channel counts are multiples of 32, at most 96, and the
 *     output channel count is 32, 64 or 96; the image width is a multiple
 *     of 64;
 *   - weights are [co][9][ci] with tap t = 3 (dy + 1) + (dx + 1); the
 *     data-gradient pass takes the flipped, transposed copy [ci][9][co]
 *     (wflip[ci][8 - t][co] = w[co][t][ci]) that nn_adam and
 *     nn_cast_weights maintain;
 *   - every call is ordered on `stream` (a hipStream_t, NULL = null stream)
 *     and returns 0 (LBM_OK) or a negative lbm_status; nothing synchronises
 *     except nn_features / nn_to_fields / nn_targets, which upload a small
 *     per-channel table first;
 *   - buffers are owned by the caller; none may alias unless stated.
 */
#ifndef LBM_NN_H
#define LBM_NN_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* y = act(conv3x3(x, w) + bias).  x [n][h][wd][ci] bf16, w [co][9][ci] bf16,
 * bias [co] float32 or NULL.  Outputs: y [n][h][wd][co] bf16 (or NULL) and/or
 * y32 [n][h][wd][y32_channels] float32 holding the first y32_channels output
 * channels (or NULL).  relu != 0 applies max(0, .). */
int nn_conv3x3_fwd(const uint16_t* x, const uint16_t* w, const float* bias, uint16_t* y, float* y32,
                   int32_t y32_channels, int32_t n, int32_t h, int32_t wd, int32_t ci, int32_t co, int32_t relu,
                   void* stream);

/* Tuning: the row-walking forward kernel (rows of 256 or 128 pixels, the
 * channel pairs of the network's two upper levels) lets one work-group walk
 * down several consecutive row steps of an image, sharing input rows.
 * steps > 0 fixes how many (used when it divides the steps of an image, else
 * 1); 0 restores the automatic choice.  Library-wide setting; results do not
 * depend on it.  LBM_EINVAL for steps < 0 or > 64. */
int nn_set_conv_walk(int32_t steps);

/* dx = gradient of the convolution with respect to its input: dy
 * [n][h][wd][co] bf16, wflip [ci][9][co] bf16, dx [n][h][wd][ci] bf16. */
int nn_conv3x3_bwd_data(const uint16_t* dy, const uint16_t* wflip, uint16_t* dx, int32_t n, int32_t h, int32_t wd,
                        int32_t ci, int32_t co, void* stream);

/* Workspace (bytes) that nn_conv3x3_bwd_weight needs for these sizes. */
int nn_conv3x3_wgrad_workspace(int32_t n, int32_t h, int32_t wd, int32_t ci, int32_t co, int64_t* bytes);

/* dw [co][9][ci] float32 = sum over pixels of dy x shifted x; db [co] float32
 * = sum of dy (db may be NULL).  accumulate != 0 adds to dw, db.  The sum
 * over pixels is split into fixed chunks added in a fixed order, so the
 * result is deterministic.  work: device buffer of at least the size that
 * nn_conv3x3_wgrad_workspace reports (LBM_EINVAL if smaller). */
int nn_conv3x3_bwd_weight(const uint16_t* x, const uint16_t* dy, float* dw, float* db, void* work, int64_t work_bytes,
                          int32_t accumulate, int32_t n, int32_t h, int32_t wd, int32_t ci, int32_t co, void* stream);

/* ReLU backward: dx[k] = dy[k] where y[k] > 0, else 0 (y the ReLU output);
 * count elements; dx may alias dy. */
int nn_relu_bwd(const uint16_t* dy, const uint16_t* y, uint16_t* dx, int64_t count, void* stream);

/* out = a + b elementwise (out may alias a or b). */
int nn_add(const uint16_t* a, const uint16_t* b, uint16_t* out, int64_t count, void* stream);

/* 2x2 average pooling between [n][h][wd][c] and [n][h/2][wd/2][c] (h, wd
 * even, c a multiple of 8, buffers 16-byte aligned; n h and wd c below
 * 2^31).  backward = 0: in is the fine tensor, out the coarse one;
 * backward = 1: in is the coarse gradient, out the fine gradient. */
int nn_pool2(int32_t backward, const uint16_t* in, uint16_t* out, int32_t n, int32_t h, int32_t wd, int32_t c,
             void* stream);

/* Nearest-neighbour x2 upsampling between [n][h][wd][c] (coarse) and
 * [n][2h][2wd][c] (c a multiple of 8, buffers 16-byte aligned; 2 n h and
 * 2 wd c below 2^31).  backward = 0: coarse -> fine; backward = 1: fine
 * gradient -> coarse gradient (sum of the four children). */
int nn_up2(int32_t backward, const uint16_t* in, uint16_t* out, int32_t n, int32_t h, int32_t wd, int32_t c,
           void* stream);

/* Mean squared error over npix pixels and nch channels of pred and target
 * ([npix][nch] float32).  loss: device float64 scalar (the mean); dpred
 * ([npix][cpad] bf16, may be NULL) receives 2 (pred - target) / (npix nch),
 * zero in channels nch .. cpad-1.  work: at least 8 * ceil(npix / 256)
 * bytes of device memory. */
int nn_mse(const float* pred, const float* target, uint16_t* dpred, int32_t cpad, int64_t npix, int32_t nch,
           double* loss, void* work, int64_t work_bytes, void* stream);

/* nn_mse without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving or training loops, harnesses that forbid hipMalloc).  Same
 * arguments, kernels and results (bit for bit) as nn_mse; the per-block
 * partial sums go to a static device array of the library (1 MiB per GPU,
 * held until the process ends), so npix is limited to 2^25 (LBM_EINVAL
 * beyond).  The first call on a device resolves that array's address (make
 * it outside a stream capture).  All calls on one GPU share the array:
 * calls that overlap in time on one GPU (two streams, two threads) race and
 * must be ordered by the caller.  LBM_EDEVICE if the array cannot be
 * resolved. */
int nn_mse_noalloc(const float* pred, const float* target, uint16_t* dpred, int32_t cpad, int64_t npix, int32_t nch,
                   double* loss, void* stream);

/* One Adam step (bias-corrected, step >= 1, decoupled weight decay) on n
 * float32 parameters w with gradient g and moments m, v.  If w16 is given
 * it receives the bf16 copy; if wflip is given (convolution weights, n =
 * co * 9 * ci) it receives the flipped copy. */
int nn_adam(float* w, uint16_t* w16, uint16_t* wflip, const float* g, float* m, float* v, int64_t n, int32_t co,
            int32_t ci, int64_t step, float lr, float beta1, float beta2, float eps, float weight_decay,
            void* stream);

/* bf16 copy and flipped copy of float32 convolution weights [co][9][ci]. */
int nn_cast_weights(const float* w, uint16_t* w16, uint16_t* wflip, int32_t co, int32_t ci, void* stream);

/* Network input of n channels of equal size (ny x nx from params[0]):
 * x [n][ny][nx][cpad] bf16 with the planes
 *   0 bottom-wall temperature minus T_ref (dT cos(2 pi x / l) + T_h - T_ref),
 *   1 cold-start phi (tanh profile of width W at y = b - 1/2),
 *   2 mu(phi) / mu_b, 3 k(phi) / k_b,
 *   4 sigma_T / 2e-4, 5 sigma_TT / 3e-4,
 *   6 (y + 1/2) / ny, 7 b / ny,
 *   8 ln(mu_a / mu_b) / ln 5, 9 ln(k_a / k_b) / ln 5 (both layers' properties
 *     everywhere, not only inside each layer),
 * zero beyond.  cpad >= 10.  Synchronises. */
int nn_features(const lbm_params* params, int32_t n, uint16_t* x, int32_t cpad, void* stream);

/* Network output pred [n][ny][nx][4] float32 (u / U_s, v / U_s,
 * (T - T_ref) / dT, 50 (phi - phi_cold) on the interface band) -> fields
 * [n][phi | ux | uy | T][ny][nx] float64 in the layout lbm_init_device
 * reads.  phi_cold is the cold-start tanh profile (width W at y = b - 1/2);
 * the band is |y - (b - 1/2)| <= 3 W.  phi_from_net == 0: phi = phi_cold.
 * phi_from_net != 0: phi = phi_cold + the predicted deviation on the band,
 * plus a rigid shift of the interface (proportional to d phi_cold / dy)
 * that makes sum phi equal the cold start's -- the conservative Allen-Cahn
 * equation keeps sum phi, so the warm and cold starts reach the same steady
 * state.  Phi outside the band is exactly phi_cold (a bulk error there
 * would decay only by diffusion at mobility M_phi).  Synchronises. */
int nn_to_fields(const lbm_params* params, int32_t n, const float* pred, double* fields, int32_t phi_from_net,
                 void* stream);

/* Training targets from converged fields: fields [n][phi | ux | uy | T]
 * [ny][nx] float64 -> target [n][ny][nx][4] float32 (u / U_s, v / U_s,
 * (T - T_ref) / dT, 50 (phi - phi_cold) on the interface band and 0
 * outside).  nn_to_fields inverts it up to float32 rounding and, for phi,
 * the sum-restoring shift.  Synchronises. */
int nn_targets(const lbm_params* params, int32_t n, const double* fields, float* target, void* stream);

/* Velocity scale U_s of the network outputs for one channel:
 * 0.01 (|sigma_T| + sigma_TT dT) dT / mu_b (at least 1e-12). */
double nn_velocity_scale(const lbm_params* p);

#ifdef __cplusplus
}
#endif

#endif /* LBM_NN_H */
