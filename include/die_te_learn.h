/*
 * die_te_learn.h -- C ABI of the learned warm start of the TE DIE solver.
 *
 * Not part of the paper's method: restarted GMRES (Section 4) may start from any
 * initial guess x0, and this part proposes one with a U-Net trained on solutions
 * the solver itself produced.  The solver's FP64 true-residual acceptance is
 * unchanged, so the guess can only change the iteration count, never the answer.
 *
 * Network (levels L >= 1, base width C >= 8, C % 8 == 0): encoder levels l = 0..L-1
 * of two 3x3 convolutions (zero padding 1) + ReLU with C 2^l channels, a 2x2 average
 * pool after every level but the last; decoder levels l = L-2..0: nearest 2x
 * upsampling, channel concatenation [upsampled, encoder output of level l], two 3x3
 * convolutions + ReLU with C 2^l channels; a 1x1 head to 4 channels.
 * Input  x: [batch][H][W][8] float32, channels Re chi, Im chi, Re E1_in, Im E1_in,
 *           Re E2_in, Im E2_in, 0, 0 (die_te_unet_pack_inputs builds it).
 * Output y: [batch][H][W][4] float32, Re/Im of the scattered field E - E_in per
 *           component (x0 = E_in + y).
 * H and W must be multiples of 8 * 2^(L-1) (the coarsest level is a multiple of 8 wide).
 *
 * Parameters: one float32 vector, layer by layer (enc0a, enc0b, ..., enc(L-1)b,
 * dec(L-2)a, dec(L-2)b, ..., dec0b, head), each layer its weights W[co][t][ci]
 * (t = 3 (dy + 1) + (dx + 1) is the tap that multiplies the input at (y + dy, x + dx);
 * t = 0 for the 1x1 head) followed by its bias[co].
 *
 * Arithmetic: convolutions on the matrix cores with bfloat16 operands (weights and
 * stored activations rounded to nearest even) and float32 accumulation; activation
 * gradients float32, rounded to bfloat16 where they enter a convolution; parameter
 * gradients, loss and Adam float32.  Sums are in a fixed order: results are
 * deterministic for a given batch.
 *
 * Conventions are those of die_te.h (device pointers, stream, return codes,
 * die_te_last_error()).  A network object is not thread safe.
 */
#ifndef DIE_TE_LEARN_H
#define DIE_TE_LEARN_H

#include "die_te.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct die_te_unet die_te_unet;

/* Allocate a network for inputs of H x W pixels and batches of at most max_batch,
 * with He-normal weights (standard deviation sqrt(2 / (taps cin)), from a seeded
 * generator) and zero biases.  Synchronises `stream`. */
int die_te_unet_create(die_te_unet **net, int levels, int base, int height, int width, int max_batch,
                       unsigned long long seed, void *stream);

/* Number of float32 parameters. */
int die_te_unet_num_params(const die_te_unet *net, long long *n);

/* Copy the parameters (host float32 [n]) out of / into the network; set also resets
 * the optimiser state.  Synchronise `stream`. */
int die_te_unet_get_params(die_te_unet *net, float *params, void *stream);
int die_te_unet_set_params(die_te_unet *net, const float *params, void *stream);

/* Copy the parameter gradient of the last die_te_unet_loss_grad (host float32 [n]). */
int die_te_unet_get_grads(die_te_unet *net, float *grads, void *stream);

/* y = network(x).  x: device float32 [batch][H][W][8]; y: device float32
 * [batch][H][W][4]; 1 <= batch <= max_batch.  Asynchronous. */
int die_te_unet_forward(die_te_unet *net, const float *x, float *y, int batch, void *stream);

/* Mean-square loss mean((network(x) - target)^2) over all batch*H*W*4 outputs and its
 * parameter gradient (kept in the network).  target: device float32 [batch][H][W][4].
 * *loss (host) receives the loss.  Synchronises `stream`. */
int die_te_unet_loss_grad(die_te_unet *net, const float *x, const float *target, int batch, double *loss,
                          void *stream);

/* One Adam step (Kingma & Ba 2015, bias-corrected moments) with the stored gradient:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).  Asynchronous. */
int die_te_unet_adam(die_te_unet *net, float lr, float beta1, float beta2, float eps, void *stream);

/* die_te_unet_loss_grad followed by die_te_unet_adam(lr, 0.9, 0.999, 1e-8). */
int die_te_unet_train_step(die_te_unet *net, const float *x, const float *target, int batch, float lr,
                           double *loss, void *stream);

/* Network input from the permittivity and the incident field (all device):
 * eps_r complex128 [nobj][ny][nx], e_in complex128 [batch][2][ny][nx]; sample r uses
 * object r / (batch / nobj) (batch a multiple of nobj); x float32 [batch][ny][nx][8]. */
int die_te_unet_pack_inputs(const void *eps_r, int nobj, const void *e_in, float *x, int batch, int ny, int nx,
                            void *stream);

/* Training target: t float32 [batch][ny][nx][4] = Re/Im of e_tot - e_in per component
 * (e_tot, e_in complex128 [batch][2][ny][nx], device). */
int die_te_unet_pack_targets(const void *e_tot, const void *e_in, float *t, int batch, int ny, int nx,
                             void *stream);

/* Initial guesses for die_te_solve: x0 = e_in + network(inputs from the context's
 * contrast and e_in) for nrhs fields of the context's grid (right-hand side r uses
 * object r / (nrhs / nobj), as in die_te_solve).  The network's H x W must equal the
 * context's ny x nx.  e_in, x0: device complex128 [nrhs][2][ny][nx].  Pass x0 to
 * die_te_solve with x0_given = 1.  Synchronises `stream`. */
int die_te_warm_start(die_te_ctx *ctx, die_te_unet *net, const void *e_in, void *x0, int nrhs, void *stream);

/* Release the network. */
int die_te_unet_destroy(die_te_unet *net);

#ifdef __cplusplus
}
#endif
#endif /* DIE_TE_LEARN_H */
