/*
 * MAGPIE learned start: C ABI of the coarse-object network, its training
 * kernels, the network input map and the whole-object pyramid.
 *
 * The paper leaves the initial guess of Alg 4 unspecified (a flat start is
 * the plain method).  This interface adds a starting guess predicted by a
 * small convolutional network; the plain method stays the fallback and
 * decides whether the guess is used (magpie_learned_start keeps whichever
 * start has the lower objective, eq. 2.1).
 *
 * Network (fixed architecture, width W = 32): five 3x3 convolutions with zero
 * padding 1: Cin -> W, ReLU, W -> W, ReLU, nearest 2x upsampling, W -> W, ReLU,
 * W -> W, ReLU, W -> 2.  Input [B][Cin][S][S] float32; output
 * [B][2][2S][2S] float32 = (log-amplitude, phase) of the coarse object.
 * Parameters are one float32 vector: per layer W_l[co][ci][3][3] then b_l[co].
 *
 * Conventions are those of magpie.h: return codes MAGPIE_OK / MAGPIE_ERR_*,
 * magpie_last_error() for the message, on_device = 1 for device pointers
 * (read in stream order on the object's stream), 0 for host pointers (copied
 * before return, outputs complete on return).  Every call is deterministic:
 * reductions run in a fixed order.
 */
#ifndef MAGPIE_LEARNED_H
#define MAGPIE_LEARNED_H

#include <stdint.h>

#include "magpie.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct magpie_cnn magpie_cnn;

#define MAGPIE_W_F32 0  /* weights used in float32 */
#define MAGPIE_W_BF16 1 /* weights rounded to bfloat16 (nearest even) for the convolutions; fp32 master copy */

#define MAGPIE_COARSE_C64 0     /* interleaved complex64 [side][side] */
#define MAGPIE_COARSE_C128 1    /* interleaved complex128 */
#define MAGPIE_COARSE_LOGPOLAR 2 /* float32 planes [2][side][side]: log-amplitude, phase (network output) */

/* Create a network on `device` for inputs of `in_ch` (1, 3 or 4) channels of
 * side x side pixels (side a multiple of 2), width 32, batches of up to
 * max_batch.  weight_dtype: MAGPIE_W_F32 or MAGPIE_W_BF16.  stream: a
 * hipStream_t or NULL (the network creates its own).  Parameters start at 0. */
int magpie_cnn_create(magpie_cnn** out, int in_ch, int width, int side, int max_batch, int weight_dtype, int device,
                      void* stream);
int magpie_cnn_destroy(magpie_cnn* net);
int magpie_cnn_num_params(const magpie_cnn* net, int64_t* n);

/* Set / read the parameter vector (n floats).  Setting resets the Adam state. */
int magpie_cnn_set_params(magpie_cnn* net, const float* params, int on_device);
int magpie_cnn_get_params(magpie_cnn* net, float* params, int on_device);
/* Gradient of the last backward pass (n floats). */
int magpie_cnn_get_grads(magpie_cnn* net, float* grads, int on_device);

/* y = net(x) for nbatch <= max_batch samples; activations are kept for
 * magpie_cnn_backward.  y may be NULL (kept internally). */
int magpie_cnn_forward(magpie_cnn* net, const float* x, float* y, int nbatch, int on_device);

/* Masked complex MSE of exp(y0 + i y1) from the last forward against
 * target (complex64 [nbatch][2S][2S]) with pixel weights mask (float
 * [2S][2S], >= 0, not all 0): sum_n sum_p mask |pred - target|^2 / (nbatch sum_p mask).
 * align_phase = 1 first rotates each sample's prediction by its best global
 * phase (the objective of eq. 2.1 is blind to it); the gradient then holds
 * that phase fixed, which is exact at the minimiser.
 * Stores dL/dy for the next backward; *loss (host) is written on return. */
int magpie_cnn_loss(magpie_cnn* net, const void* target, const float* mask, int nbatch, int align_phase,
                    int on_device, double* loss);

/* Parameter gradient of sum(dy * y) for the last forward.  dy: [nbatch][2][2S][2S],
 * or NULL to use the gradient stored by magpie_cnn_loss. */
int magpie_cnn_backward(magpie_cnn* net, const float* dy, int nbatch, int on_device);

/* One Adam step (bias-corrected, Kingma and Ba 2015) on the last gradient. */
int magpie_cnn_adam_step(magpie_cnn* net, float lr, float beta1, float beta2, float eps);

int magpie_cnn_sync(magpie_cnn* net);

/* Network input map of a reconstruction context (needs probe, positions and
 * intensities): per position k, a_k = mean sqrt(d_k) / ||Q||_2 and the centre
 * of mass of d_k over signed frequency indices (rows, then columns); each is
 * spread over the object with weights |Q(p - o_k)|^2, normalised per pixel
 * (0 where no position covers p), then averaged over
 * (n_rows / side) x (n_cols / side) blocks; channel 3 is the phase those
 * centres of mass integrate to (a centre of mass of f bins is a phase slope of
 * 2 pi f / m per object pixel), least-squares over the whole map (spectral,
 * periodic, mean 0).  out: float [4][side][side].  side must divide n_rows and
 * n_cols and be at most 64. */
int magpie_input_map(magpie_ctx* ctx, int side, float* out, int on_device);

/* Object <- (I_H^h)^j applied to a coarse object (eq. 2.6: each coarse value
 * copied into its f x f block, f = n_rows / side = n_cols / side = 2^j).
 * format: MAGPIE_COARSE_*. */
int magpie_set_object_from_coarse(magpie_ctx* ctx, const void* coarse, int side, int format, int on_device);

/* out = (I_h^H)^j z on the whole object (eq. 2.5: f x f block means,
 * f = 2^times), complex64 in and out, device pointers, on `stream`. */
int magpie_restrict_object(const void* z, int n_rows, int n_cols, int times, void* out, void* stream);

/* Learned start: input map -> network -> coarse object -> prolongation;
 * then the objective of the learned start and of the flat start (all ones)
 * are evaluated and the lower one is kept as the object.  *used = 1 if the
 * learned start was kept.  phi_learned / phi_flat / used may be NULL.
 * The network reads the map's first in_ch channels (1, 3 or 4), and side such
 * that 2 * side divides the object and the ratio is a power of two. */
int magpie_learned_start(magpie_ctx* ctx, magpie_cnn* net, double* phi_learned, double* phi_flat, int* used);

#ifdef __cplusplus
}
#endif

#endif /* MAGPIE_LEARNED_H */
