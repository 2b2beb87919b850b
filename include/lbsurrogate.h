/* C ABI of the learned surrogate of the lattice Boltzmann step (BF16 matrix
 * cores, FP32 accumulation), built into liblbvdw.so beside include/lbvdw.h.
 *
 * The paper has no surrogate: this is an accelerator placed around its
 * method. A small convolutional network predicts the change of the fields
 * (n, u*_x, u*_y) over a chunk of lattice steps; the lattice itself audits
 * the predictions (lb_batch_step_subset on a rotating subset of instances)
 * and replaces rejected ones; accepted ones re-enter the lattice through
 * the change of the equilibrium populations of Eq.(eqfunc)
 * (lb_batch_shift_equilibrium_device) or as those equilibria
 * (lb_batch_set_equilibrium_device).
 *
 * Network (fixed shape): 3x3 convolutions, x periodic, zero padding beyond
 * the first and last rows;
 *   h0 = SiLU(conv(x) + b0)                  LBS_IN_REAL -> LBS_WIDTH channels
 *   h_l = h_{l-1} + SiLU(conv(h_{l-1}) + b_l) l = 1..LBS_BLOCKS, LBS_WIDTH -> LBS_WIDTH
 *   out = conv(h_LBS_BLOCKS) + b_out         LBS_WIDTH -> LBS_OUT
 * Activations are bf16, accumulation and the output are FP32, master
 * parameters FP32. Parameter vector (FP32), layer after layer: weights
 * w[tap][ci][co] with tap = 3 (dy + 1) + (dx + 1), then biases b[co], with
 * the real channel counts above.
 *
 * Tensors are NHWC: [batch][H rows (y)][W columns (x)][channels]. Network
 * inputs are bf16 with LBS_IN_CHANNELS channels (the last two zero), outputs
 * FP32 with LBS_OUT channels. All tensor pointers are device pointers owned
 * by the caller, 16-byte aligned; calls are asynchronous on the given HIP
 * stream unless stated. Errors: LB_EINVAL for bad sizes, shapes or NULL
 * pointers (checked before any device work), LB_ENOMEM for a workspace that
 * is too small, LB_EDEVICE for HIP failures; lb_last_error() describes the
 * last failure of the calling thread. */
#ifndef LBSURROGATE_H
#define LBSURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "lbvdw.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBS_IN_CHANNELS 8
#define LBS_IN_REAL 6
#define LBS_WIDTH 48
#define LBS_BLOCKS 4
#define LBS_OUT 3
#define LBS_OUT_CHANNELS 16 /* padded output channels of the last layer's gradient */

typedef struct lbs_net lbs_net;

/* Scalings between lattice fields and network tensors. Input channels:
 * (n - 1) n_scale, u*_x u_scale, u*_y u_scale, V(x) v_scale (V the external
 * force density of the column, paper units), wall speed u_scale on the wall
 * rows (-U on row 0, +U on row H - 1, zero elsewhere and in periodic runs),
 * (T - 0.9) t_scale, 0, 0. Output channels: the change of n, u*_x, u*_y over
 * one chunk times n_scale, u_scale, u_scale. */
typedef struct {
  float n_scale, u_scale, v_scale, t_scale;
} lbs_scales;

/* Number of FP32 parameters of the network. */
lb_status lbs_param_count(int64_t* count);

/* Device workspace of a network for batches of up to max_batch images of
 * H x W (train != 0: also gradients, Adam moments and the activations the
 * backward pass needs). */
lb_status lbs_workspace_bytes(int32_t max_batch, int32_t H, int32_t W, int32_t train,
                              size_t* bytes);

/* Create a network in a caller-owned device workspace (256-byte aligned,
 * lbs_workspace_bytes long) on a caller stream (NULL = the null stream).
 * Parameters start at zero: set them with lbs_set_params. */
lb_status lbs_create(int32_t max_batch, int32_t H, int32_t W, int32_t train, void* dev_ws,
                     size_t ws_bytes, void* hip_stream, lbs_net** out);

/* Copy FP32 parameters (device, lbs_param_count values) into the network;
 * resets the Adam moments and step counter. */
lb_status lbs_set_params(lbs_net* net, const float* d_params);
/* Copy the FP32 parameters out (device). */
lb_status lbs_get_params(lbs_net* net, float* d_params);

/* Inference: d_x [B][H][W][LBS_IN_CHANNELS] bf16 -> d_out [B][H][W][LBS_OUT]
 * FP32, 1 <= B <= max_batch. When W is a multiple of 64 the LBS_BLOCKS
 * residual layers run as one pass over HBM (their activations stay on chip);
 * the result is the same bits as running them layer by layer. */
lb_status lbs_forward(lbs_net* net, int32_t B, const void* d_x, float* d_out);

/* One training step on a batch: forward, loss = mean over nodes and the
 * LBS_OUT channels of (out - target)^2, backward, Adam (Kingma and Ba; beta1
 * 0.9, beta2 0.999, eps 1e-8, learning rate lr). d_target [B][H][W][LBS_OUT]
 * FP32. Writes the loss before the update to d_loss (device FP64, may be
 * NULL). Requires train != 0 at create. */
lb_status lbs_train_step(lbs_net* net, int32_t B, const void* d_x, const float* d_target, float lr,
                         double* d_loss);

/* The FP32 gradient of the last lbs_train_step (device, lbs_param_count). */
lb_status lbs_get_grads(lbs_net* net, float* d_grads);

lb_status lbs_destroy(lbs_net* net);

/* ---- layers (the kernels the network runs), for tests and for callers
 * composing their own networks of these shapes. Supported channel pairs
 * (ci, co) of lbs_conv: (8, 48), (48, 48), (48, 16), (16, 48); of
 * lbs_wgrad: (8, 48), (48, 48), (48, 16). ---- */

/* Pack FP32 weights w[9][cir][cor] into the bf16 matrix a convolution
 * kernel reads. transposed = 0: for a ci -> co convolution with ci = CI,
 * co = CO (padded counts, cir <= CI, cor <= CO), [CO][k], k = tap CI + ci.
 * transposed = 1: for the input gradient (a CO -> CI convolution with the
 * taps flipped), [CI][k], k = tap' CO + co, holding w[8 - tap'][ci][co].
 * k is zero-padded to a multiple of 32. wpack holds
 * rows x ceil(9 kin / 32) 32 values, rows = CO or CI, kin = CI or CO. */
lb_status lbs_pack(const float* d_w, int32_t cir, int32_t cor, int32_t CI, int32_t CO,
                   int32_t transposed, void* d_wpack, void* hip_stream);

/* One 3x3 convolution of x [B][H][W][ci] (bf16) with packed weights; the
 * epilogue depends on mode:
 *   0 first layer: v = conv + bias; y = SiLU(v), z = v (bf16; z may be NULL)
 *   1 residual:    v = conv + bias; y = res + SiLU(v), z = v
 *   2 output:      yf[..][c] = conv + bias for c < nout (FP32 [B][H][W][nout])
 *   3 backward:    g = conv + res (res may be NULL); z = g (may be NULL),
 *                  y = g SiLU'(zprev)   (x holds dL/dz of the layer above and
 *                  the weights are packed transposed)
 * bias: FP32 [co] (first / residual) or [nout] (output), may be NULL; the
 * backward mode takes none (LB_EINVAL otherwise). The products
 * accumulate in FP32 starting from the bias; in mode 1 the residual is added
 * in the rounding of SiLU's product (one fused multiply-add).
 * The kernel is persistent: each workgroup walks 8-row x 64-column tiles
 * (stride: the grid). blocks caps the grid (0: one workgroup per tile, at
 * most as many as fit on the device at once; 1 <= blocks <= 4096 forces a
 * smaller grid, so that every workgroup walks several tiles). Results do not
 * depend on the grid. */
lb_status lbs_conv(int32_t mode, int32_t ci, int32_t co, const void* d_x, const void* d_wpack,
                   const float* d_bias, const void* d_res, const void* d_zprev, void* d_y,
                   void* d_z, float* d_yf, int32_t nout, int32_t B, int32_t H, int32_t W,
                   int32_t blocks, void* hip_stream);

/* Weight and bias gradients: dw[tap][ci][co] (ci < cir, co < cor; FP32) =
 * scale * sum over pixels p of x[p + offset(tap)][ci] gz[p][co], with the
 * convolution's boundary rules, and db[co] = scale * sum_p gz[p][co] (db may
 * be NULL); x [B][H][W][ci], gz [B][H][W][co] bf16. d_part: scratch of
 * lbs_wgrad_scratch_floats FP32 values (per-workgroup partial sums, added in
 * a fixed order, so results are deterministic); 1 <= blocks <= 4096
 * workgroups. */
lb_status lbs_wgrad_scratch_floats(int32_t ci, int32_t co, int32_t cir, int32_t cor, int32_t blocks,
                                   int64_t* count);
lb_status lbs_wgrad(int32_t ci, int32_t co, int32_t cir, int32_t cor, const void* d_x,
                    const void* d_gz, int32_t B, int32_t H, int32_t W, float scale, float* d_part,
                    int32_t blocks, float* d_dw, float* d_db, void* hip_stream);

/* lbs_wgrad without a caller scratch, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc). Same arguments, kernels and results as lbs_wgrad, with
 * the per-workgroup partial sums in a static device array of 4 Mi floats
 * (16 MiB, one per GPU, held until the process ends). LB_EINVAL when
 * lbs_wgrad_scratch_floats(ci, co, cir, cor, blocks) exceeds it (for
 * (48, 48, 48, 48), blocks <= 169). The call allocates nothing. Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller. */
lb_status lbs_wgrad_noalloc(int32_t ci, int32_t co, int32_t cir, int32_t cor, const void* d_x,
                            const void* d_gz, int32_t B, int32_t H, int32_t W, float scale,
                            int32_t blocks, float* d_dw, float* d_db, void* hip_stream);

/* Bias gradient db[c] = scale * sum_p gz[p][c] for c < nreal; gz [npix][C]
 * bf16, C <= 64; d_part: 1024 C FP32 of scratch. */
lb_status lbs_bias_grad(const void* d_gz, int64_t npix, int32_t C, int32_t nreal, float scale,
                        float* d_part, float* d_db, void* hip_stream);

/* Loss: *d_loss = mean over npix nodes and nout channels of (pred - target)^2
 * (FP64 sums); d_gout [npix][CO] bf16 = 2 (pred - target), zero for c >= nout.
 * d_part: 512 FP64 of scratch. */
lb_status lbs_mse(const float* d_pred, const float* d_target, int64_t npix, int32_t nout,
                  int32_t CO, void* d_gout, double* d_part, double* d_loss, void* hip_stream);

/* Adam step t (>= 1) on n FP32 parameters. */
lb_status lbs_adam(float* d_p, const float* d_g, float* d_m, float* d_v, int32_t n, float lr,
                   float beta1, float beta2, float eps, int32_t t, void* hip_stream);

/* ---- fields <-> network tensors, batched over B instances of H x W nodes.
 * Field blocks are device FP64 [B][3][H][W] (n, u*_x, u*_y), the layout of
 * lb_batch_get_moments_device. ---- */

/* Network input of the fields. d_vx: FP32 [B][W] external force density per
 * column (paper units); d_cond: FP32 [B][2] (wall speed U, temperature T);
 * walls != 0 for runs with walls. */
lb_status lbs_fields_to_input(const double* d_fields, int32_t B, int32_t H, int32_t W,
                              const float* d_vx, const float* d_cond, int32_t walls,
                              const lbs_scales* s, void* d_x, void* hip_stream);

/* Training target: the scaled change d_f1 - d_f0 as FP32 [B][H][W][3]. */
lb_status lbs_make_target(const double* d_f0, const double* d_f1, int32_t B, int64_t nn,
                          const lbs_scales* s, float* d_target, void* hip_stream);

/* Predicted fields d_f1 = d_f0 + out / scales (FP64). */
lb_status lbs_apply_output(const double* d_f0, const float* d_out, int32_t B, int64_t nn,
                           const lbs_scales* s, double* d_f1, void* hip_stream);

/* Per instance b (FP64, fixed order): d_out[6b..6b+5] = (sum n_a, sum n_b,
 * max over nodes |n_a - n_b| / n_b, number of nodes with n_a not finite or
 * outside (0, 3), sum (n_a - n_b)^2, sum n_b^2). */
lb_status lbs_compare(const double* d_a, const double* d_b, int32_t B, int64_t nn, double* d_out,
                      void* hip_stream);

/* Mass projection: for instances with d_mask[b] != 0 (device int32), add the
 * uniform shift (sum n_ref - sum n_a) / nn to n_a. */
lb_status lbs_project_mass(double* d_a, const double* d_ref, int32_t B, int64_t nn,
                           const int32_t* d_mask, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBSURROGATE_H */
