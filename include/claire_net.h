/*
 * Learned warm start for the Gauss--Newton--Krylov registration solve: a
 * periodic 3D convolutional encoder--decoder that predicts an initial
 * velocity from (m0, m1). The solver keeps the final word: the prediction is
 * only the starting point v0 of claire_ctx_solve / claire_solve (Alg. 1),
 * the same hook the paper's parameter continuation uses when each level
 * starts from the previous level's solution (Section 2.6). The network
 * itself is not part of the paper.
 *
 * Network (working resolution R^3, R a power of two >= 8, channels
 * c1..c4 multiples of 8):
 *   input   8 channels (m0, m1, m1 - m0, 0 x 5), channels last;
 *   conv    3x3x3, periodic wrap, cross-correlation
 *           y(i, co) = b(co) + sum_t sum_ci w(co, t, ci) x(i + o_t, ci),
 *           tap t = 9 (o1 + 1) + 3 (o2 + 1) + (o3 + 1), o in {-1, 0, 1}^3;
 *   act     LeakyReLU(0.1) after every conv but the last;
 *   encoder two convs per level at R, R/2, R/4, R/8 (c1..c4 channels),
 *           2x2x2 average pooling between levels;
 *   decoder nearest 2x upsampling, concatenation [upsampled, encoder skip],
 *           two convs per level; a last conv to 3 channels gives v;
 *   loss    mean squared error against a target velocity; Adam optimiser.
 * Parameters (float32, flat): per layer, in the order enc1a enc1b enc2a
 * enc2b enc3a enc3b bota botb dec3a dec3b dec2a dec2b dec1a dec1b head, the
 * weights w[co][t][ci] (C order) followed by the biases b[co].
 * Precision: every convolution operand (input features, stored activations,
 * gradients w.r.t. pre-activations, weights) is bfloat16 (round to nearest
 * even); products accumulate in float32 on the matrix cores; master
 * weights, Adam moments, the output v and all other arithmetic are float32.
 *
 * All array arguments are device pointers (16-byte aligned) unless stated;
 * fields are channels first, x3 fastest: images [batch][R^3], velocities
 * [batch][3][R^3] or [3][n]. Calls enqueue on the stream given at creation
 * and return 0 or a negative CLAIRE_E* code with claire_last_error() set.
 */
#ifndef CLAIRE_NET_H
#define CLAIRE_NET_H

#include "claire.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct claire_net claire_net;

/* Create a network for working resolution res^3 (power of two, 8..256),
 * channels c[4] (multiples of 8, at most 256), batches up to max_batch.
 * Weights start at He-uniform values from `seed` (biases zero).
 * CLAIRE_EINVAL on bad sizes, CLAIRE_ENOMEM if device memory runs out. */
int claire_net_create(claire_net** out, int res, const int channels[4], int max_batch,
                      unsigned long long seed, void* stream);
int claire_net_destroy(claire_net* net);

/* Number of float32 parameters (layout above). */
long long claire_net_param_count(const claire_net* net);

/* Copy the parameters in or out (device float32[param_count]). Setting them
 * resets the Adam state. */
int claire_net_set_params(claire_net* net, const float* params);
int claire_net_get_params(const claire_net* net, float* params);
/* Gradient of the last claire_net_loss_grad / claire_net_train_step. */
int claire_net_get_grads(const claire_net* net, float* grads);
/* Replace the kept gradient (device float32[param_count]), e.g. to apply
 * claire_net_adam_step to a gradient computed elsewhere. */
int claire_net_set_grads(claire_net* net, const float* grads);

/* v [batch][3][R^3] = network(m0, m1), images [batch][R^3]. */
int claire_net_forward(claire_net* net, const float* m0, const float* m1, int batch,
                       float* v);

/* Forward, mean-squared-error loss against v_target [batch][3][R^3] (host
 * double *loss, synchronises the stream) and the parameter gradient, kept in
 * the network. v (nullable) receives the prediction. */
int claire_net_loss_grad(claire_net* net, const float* m0, const float* m1,
                         const float* v_target, int batch, double* loss, float* v);

/* One Adam step (b1 0.9, b2 0.999, eps 1e-8, bias corrected) with the kept
 * gradient and learning rate lr. */
int claire_net_adam_step(claire_net* net, double lr);

/* loss_grad followed by adam_step. */
int claire_net_train_step(claire_net* net, const float* m0, const float* m1,
                          const float* v_target, int batch, double lr, double* loss);

/* Initial velocity v0 [3][n^3] for images m0, m1 [n^3] on the registration
 * grid (cubic, n a power of two >= R): 2x2x2 block-mean restriction to R^3,
 * the network, and periodic cubic Lagrange prolongation back to n^3. The net
 * keeps about 6 n^3 + 4 R^3 floats of scratch after the first call at a
 * given n (freed with the net). */
int claire_net_warm_start(claire_net* net, const float* m0, const float* m1, int n, float* v0);

/* Grid transfer between cubic grids by powers of two for ncomp fields
 * [ncomp][n^3]: n_dst < n_src averages 2x2x2 blocks per halving, n_dst > n_src
 * refines with the separable periodic cubic Lagrange midpoint rule
 * (-f(i-1) + 9 f(i) + 9 f(i+1) - f(i+2)) / 16 per doubling (x1, then x2, then
 * x3). src and dst must not overlap. Enqueued on `stream`. */
int claire_resample(const float* src, int n_src, float* dst, int n_dst, int ncomp,
                    void* stream);

/* One convolution layer of the network on its own, for checks: x
 * [batch][R^3][cin] float32 (rounded to bfloat16 on the way in), w
 * [cout][27][cin], b [cout] float32 (w rounded to bfloat16), y
 * [batch][R^3][cout] float32 = conv (act = 0) or LeakyReLU(conv) (act = 1),
 * not rounded. cin a multiple of 8. The network's kernels for the shape run,
 * reduction splits of small grids included. */
int claire_conv3d(const float* x, const float* w, const float* b, int batch, int res,
                  int cin, int cout, int act, float* y, void* stream);

/* Backward pass of one layer for the loss sum(dz * conv(x)), for checks:
 * dz [batch][R^3][cout] float32 (rounded to bfloat16, like x and w), dx
 * [batch][R^3][cin], dw [cout][27][cin], db [cout] float32. cout a multiple
 * of 8. */
int claire_conv3d_backward(const float* x, const float* w, const float* dz, int batch, int res,
                           int cin, int cout, float* dx, float* dw, float* db, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CLAIRE_NET_H */
