/*
 * ri_cnn.h -- C ABI of the residual CNN denoiser in libri.so (HIP, gfx950).
 *
 * The learned denoiser of the plug-and-play loop (Dabbech et al.,
 * appendix C): D(z) = z - net(z), net a stack of L 3x3 "same" convolutions
 * with biases and ReLU between them (1 -> C -> ... -> C -> 1 channels, no
 * normalisation), trained with the l1 loss E||D(u + sigma n) - u||_1 of
 * eq. (C1) (its firm-nonexpansiveness penalty is not implemented here). The
 * denoiser is applied to image facets independently (appendix D).
 *
 * Precision: the input, the first layer and the residual subtraction are
 * FP32; hidden activations and the weights of layers 2..L are bfloat16
 * (round to nearest even) with FP32 accumulation in MFMA; the last layer
 * accumulates in FP32. Gradients are FP32 (hidden pre-activation gradients
 * stored as bfloat16).
 *
 * Parameter vector (FP32, device): for each layer l = 0..L-1 its weights
 * W_l[c_out][c_in][3][3] then its biases b_l[c_out], layers in order.
 * Images are FP32 [batch][h][w] row-major; h and w multiples of 16.
 * Buffers marked "dev" are caller-owned device memory; the network object
 * owns its parameters, optimizer state and activations.
 */
#ifndef RI_CNN_H
#define RI_CNN_H

#include <stdint.h>

#include "ri.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ri_cnn ri_cnn;

typedef struct {
    int32_t layers;     /* L >= 3 */
    int32_t channels;   /* hidden channels; must be 64 */
    int32_t max_batch;  /* largest batch the activation buffers hold */
    int32_t max_h, max_w;  /* largest image side; multiples of 16 */
    int32_t training;   /* 1: keep every layer's activations and the optimizer state */
} ri_cnn_desc;

/* Create a network with He-normal weights drawn from a counter-based generator
 * seeded by `seed`, zero biases. Synchronous. */
ri_status ri_cnn_create(const ri_cnn_desc *desc, uint64_t seed, ri_cnn **out);
void ri_cnn_destroy(ri_cnn *net);
const char *ri_cnn_last_error(const ri_cnn *net);
int64_t ri_cnn_param_count(const ri_cnn *net);

/* Copy the FP32 parameter vector in (dev, param_count floats) or out. */
ri_status ri_cnn_set_params(ri_cnn *net, const float *params, ri_stream stream);
ri_status ri_cnn_get_params(const ri_cnn *net, float *params, ri_stream stream);

/* out = D(z) = z - net(z). z, out: dev [batch][h][w]. */
ri_status ri_cnn_forward(ri_cnn *net, const float *z, float *out, int32_t batch, int32_t h, int32_t w,
                         ri_stream stream);

/* Gradient of sum(g * net(z)) with respect to the parameters (FP32, the
 * parameter layout), overwriting grads (dev, param_count floats). Requires
 * training = 1. g: dev [batch][h][w]. */
ri_status ri_cnn_grad(ri_cnn *net, const float *z, const float *g, int32_t batch, int32_t h, int32_t w,
                      float *grads, ri_stream stream);

/* A training batch drawn from a pool of clean patches resident on the device:
 * out[b] = patch p_b of pool in orientation o_b, one of the eight symmetries
 * of the square (transpose, row reversal, column reversal), with (p_b, o_b)
 * from a counter-based generator keyed by (seed, b). pool: dev
 * [n_pool][side][side] FP32; out: dev [batch][side][side]. The network is
 * only used for its error message. */
ri_status ri_cnn_sample_batch(ri_cnn *net, const float *pool, int64_t n_pool, int32_t side, int32_t batch,
                              uint64_t seed, float *out, ri_stream stream);

/* One training step: noisy = clean + sigma n with n ~ N(0,1) from a
 * counter-based generator keyed by (seed, pixel index), D(noisy), loss
 * mean|D - clean| (FP64, written to loss if non-NULL, dev double[1]),
 * gradients, one Adam update (beta1 0.9, beta2 0.999, eps 1e-8) with rate lr. */
ri_status ri_cnn_train_step(ri_cnn *net, const float *clean, int32_t batch, int32_t h, int32_t w, float sigma,
                            uint64_t seed, float lr, double *loss, ri_stream stream);

/* Jacobian of the network at z (appendix C: the firm-nonexpansiveness
 * condition of the training loss asks ||J_{2D - I}||_S <= 1; these calls
 * measure it). A ReLU network is piecewise linear: at z each layer acts as its
 * convolution without bias followed by the mask [pre-activation > 0]. All
 * three run forward(z) first and need training = 1 (stored activations);
 * tangents and adjoints pass through bfloat16 like the activations and
 * gradients. z, v, u, out: dev [batch][h][w] FP32. */
/* out = J_net(z) v */
ri_status ri_cnn_jvp(ri_cnn *net, const float *z, const float *v, float *out, int32_t batch, int32_t h, int32_t w,
                     ri_stream stream);
/* out = J_net(z)^T u (the gradient of sum(u * net) with respect to z) */
ri_status ri_cnn_vjp(ri_cnn *net, const float *z, const float *u, float *out, int32_t batch, int32_t h, int32_t w,
                     ri_stream stream);
/* *norm_out (host) = ||I - 2 J_net(z)||_S = ||J_{2D - I}(z)||_S estimated by
 * iters >= 1 power iterations on J^T J from a seeded normal start (FP64
 * norms); for batch > 1 the largest over the items. Synchronous. */
ri_status ri_cnn_fne_norm(ri_cnn *net, const float *z, int32_t batch, int32_t h, int32_t w, int32_t iters,
                          uint64_t seed, double *norm_out, ri_stream stream);

/* Gradient of u^T J_net(z) v with respect to the parameters into grads (dev,
 * param_count floats; the bias entries are 0). With the ReLU masks of z fixed,
 * J_net(z) v is linear in each layer's weights, so this is the parameter
 * gradient pass run with the tangents of v as layer inputs. */
ri_status ri_cnn_jvp_grad(ri_cnn *net, const float *z, const float *v, const float *u, int32_t batch, int32_t h,
                          int32_t w, float *grads, ri_stream stream);

/* One training step with the relaxed firm-nonexpansiveness penalty (appendix
 * C; the paper relaxes the constraint of its training loss into a soft
 * penalty whose form it does not give): loss mean|D(u + sigma n) - u| +
 * lambda max(||J_{2D - I}(z)||_S^2, 1 - eps), the norm estimated by
 * power_iters iterations on J^T J warm-started from the previous call's
 * vector (a seeded normal at the first call), the penalty's gradient through
 * ri_cnn_jvp_grad's pass, one Adam update. The Jacobian is taken at
 * z = u + sigma n (point RI_FNE_AT_INPUT) or at z = rho u + (1 - rho)
 * D(u + sigma n), rho uniform in [0, 1) per batch item from the seed
 * (RI_FNE_AT_MIX: points between the clean images and their denoised versions,
 * the sampling of the relaxed scheme the paper cites). loss, fne_sq: optional
 * dev double[1] (the l1 term, and the squared norm estimate). */
enum { RI_FNE_AT_INPUT = 0, RI_FNE_AT_MIX = 1 };
ri_status ri_cnn_train_step_fne(ri_cnn *net, const float *clean, int32_t batch, int32_t h, int32_t w, float sigma,
                                uint64_t seed, float lr, float lambda, float eps, int32_t power_iters, int32_t point,
                                double *loss, double *fne_sq, ri_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* RI_CNN_H */
