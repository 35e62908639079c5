/*
 * lbm_mlp.h -- C ABI of the boiling-curve surrogate: an ensemble of small MLPs
 * (4 -> 128 -> 128 -> 2, GELU) that maps a pool-boiling configuration (wall superheat,
 * nucleation-site spacing, wall strength G_w0 of Eq. 10, gravity g of Eq. 9, each
 * scaled to [-1, 1] by the caller) to the time-averaged bottom heat flux and its
 * variance (standardised by the caller), trained on runs of the LB method.
 *
 * Arithmetic: weights and activations enter every layer product as BF16 and the
 * products accumulate in FP32 on the matrix cores (v_mfma_f32_16x16x32_bf16); biases,
 * GELU, the loss, the gradients of the biases and the Adam update are FP32; master
 * weights and Adam moments are FP32.  GELU is the exact form 0.5 z (1 + erf(z/sqrt 2)).
 * Loss per member: mean over the batch of the squared error summed over the 2 outputs.
 *
 * Host parameter layout per member (lbm_mlp_params() floats, row-major):
 *   W1[4][128], b1[128], W2[128][128], b2[128], W3[128][2], b3[2]
 * (layer l computes z = h W_l + b_l for a row vector h).  Arrays of all members are
 * consecutive.  Device arrays passed in are caller-owned; the library never allocates.
 * Every call enqueues on the stream given at init and returns LBM_OK or a negative
 * status from lbm_api.h; calls that return host data synchronise the stream.
 */
#ifndef LBM_MLP_H
#define LBM_MLP_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_MLP_IN 4
#define LBM_MLP_HIDDEN 128
#define LBM_MLP_OUT 2

typedef struct lbm_mlp lbm_mlp;

/* Parameters of one member (17410). */
size_t lbm_mlp_params(void);

/* Device workspace for `members` (1..16) networks and batches of up to max_batch rows
 * (1..1048576); 0 if out of range. */
size_t lbm_mlp_workspace_bytes(int members, int max_batch);

/* d_workspace: 256-byte aligned device memory of lbm_mlp_workspace_bytes bytes, borrowed
 * until lbm_mlp_destroy.  Parameters start at zero; set them with lbm_mlp_set_params. */
int lbm_mlp_init(int members, int max_batch, void *d_workspace, size_t ws_bytes, void *hip_stream,
                 lbm_mlp **out);

/* Load FP32 master weights (host array, members * lbm_mlp_params() floats) and reset
 * the Adam state. */
int lbm_mlp_set_params(lbm_mlp *m, const float *host);
int lbm_mlp_get_params(lbm_mlp *m, float *host);

/* d_x: device [B][4] FP32 inputs; d_y: device [members][B][2] FP32 outputs. */
int lbm_mlp_forward(lbm_mlp *m, const float *d_x, int B, float *d_y);

/* Allocation-free forward pass, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight inference loops, harnesses that forbid hipMalloc).  Same
 * arguments and results as lbm_mlp_forward (the outputs are identical), but the
 * activations go to a file-scope device array of the library, of fixed size, instead
 * of the context's workspace; the call allocates nothing (no hipMalloc, no hipFree, no
 * allocating library routine).  members * B must not exceed LBM_MLP_NOALLOC_MAX_ROWS
 * (LBM_EINVAL otherwise; the array holds 576 bytes per row, 4.5 MiB in all, on every
 * device the library runs on until the process ends).  Every call on one device shares
 * that array and leaves it holding its activations: calls that overlap on one device
 * (other streams, other host threads) race and must be ordered by the caller.  The
 * device is the one current at lbm_mlp_init, which resolves the array's address. */
#define LBM_MLP_NOALLOC_MAX_ROWS 8192
int lbm_mlp_forward_noalloc(lbm_mlp *m, const float *d_x, int B, float *d_y);

/* Forward and backward pass of every member: d_x device [B][4] inputs and d_t device
 * [B][2] FP32 targets shared by all members (per_member = 0), or [members][B][4] and
 * [members][B][2] with a batch of its own for each member (per_member = 1, e.g.
 * bootstrap resamples).  Gradients of each member's loss go to the library's gradient
 * buffers, the losses to d_loss (device, members floats). */
int lbm_mlp_backward(lbm_mlp *m, const float *d_x, const float *d_t, int B, int per_member, float *d_loss);

/* Copy the gradients of the last lbm_mlp_backward to the host (host parameter layout). */
int lbm_mlp_get_grads(lbm_mlp *m, float *host);

/* One Adam step (bias-corrected, step count kept by the library) with the stored
 * gradients; refreshes the BF16 weight copies. */
int lbm_mlp_adam(lbm_mlp *m, float lr, float beta1, float beta2, float eps);

int lbm_mlp_destroy(lbm_mlp *m);

#ifdef __cplusplus
}
#endif
#endif
