/* Learned basis surrogate of libhplmm: a small 3D convolutional network that
 * predicts grain basis columns (Eq. 23: the grain-interior response
 * -A_gi^-1 Abar_gi,m e_k to one mortar mode) from the assembled operator,
 * trained on the columns the method itself computes, with the exact local
 * solve as fallback.
 *
 * Network.  Input: 4 channels on the 9 x 9 x 9 node lattice of an 8^3-voxel
 * box grain (interior indicator; log trace of the node's diagonal 3x3 block
 * of A minus its grain mean; stored blocks of the node row / 27; the Gaussian
 * weight H_c[., a] of Eq. 8 on the nodes of interface c).  Output: 9 channels
 * = the shape vectors p_k = -A_gi^-1 Abar_gi,m e_k (Eq. 23) of the columns
 * k = 3a + x, 3a + y, 3a + z, as (u_x, u_y, u_z) each.
 * Layers: channels c0 -> c1 -> c2 -> c3 -> c4 (normally 4, 32, 32, 32, 9;
 * every c <= 32), 3x3x3 'same' convolutions with zero padding and bias, ReLU
 * after the first three.  Tensors are float32 device arrays, channel-last:
 * t[s][p][c], p = (z * 9 + y) * 9 + x.  Parameters: per layer w[d][ci][co]
 * (d = (dz+1) * 9 + (dy+1) * 3 + (dx+1)) then b[co], layers concatenated.
 *
 * Errors follow hplmm.h (status codes, hplmm_last_error()).
 */
#ifndef HPLMM_SURROGATE_H
#define HPLMM_SURROGATE_H

#include "hplmm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hplmm_sg_net hplmm_sg_net;

/* Create a network with channels[0..4] and room for batches of up to
 * max_batch samples (activations, gradients and partial sums are allocated
 * here, about 1.1 MB per sample).  Parameters start at zero.
 * E_ARG on bad channel counts or max_batch < 1; E_OOM / E_HIP. */
hplmm_status hplmm_sg_create(const int32_t channels[5], int32_t max_batch, hplmm_sg_net **out);

/* Number of float32 parameters. */
hplmm_status hplmm_sg_param_count(const hplmm_sg_net *net, int64_t *count);

/* Copy parameters from / to host memory (count must equal the parameter
 * count).  set_params also resets the Adam state. */
hplmm_status hplmm_sg_set_params(hplmm_sg_net *net, const float *host, int64_t count);
hplmm_status hplmm_sg_get_params(const hplmm_sg_net *net, float *host, int64_t count);

/* y_dev[n][729][c4] = network(x_dev[n][729][c0]); 1 <= n <= max_batch.
 * Asynchronous on stream. */
hplmm_status hplmm_sg_forward(hplmm_sg_net *net, const float *x_dev, int32_t n, float *y_dev, void *stream);

/* Inference precision of hplmm_sg_forward and of the predictions of
 * hplmm_setup_surrogate: 32 (default) = float32 operands; 16 = every layer's
 * staged inputs and weights rounded to bfloat16 (to nearest even) on the
 * matrix cores (v_mfma_f32_16x16x32_bf16), float32 accumulation, bias, ReLU
 * and activations.  Training (hplmm_sg_gradient) stays float32.  E_ARG on
 * another value. */
hplmm_status hplmm_sg_set_inference_precision(hplmm_sg_net *net, int32_t precision);

/* Forward pass, loss and gradients of the loss w.r.t. every parameter for
 * the batch (x_dev as above, y_dev the targets [n][729][c4]).  Loss = mean
 * over samples of |m (net(x) - y)|^2 / (|m y|^2 + 1e-30), m = interior
 * indicator x[s][p][0] > 0.5.  The gradients stay in the network (see
 * get_grads / adam); *loss receives the mean (synchronises the stream). */
hplmm_status hplmm_sg_gradient(hplmm_sg_net *net, const float *x_dev, const float *y_dev, int32_t n, double *loss,
                               void *stream);

/* Copy the last gradients to host memory (count = parameter count). */
hplmm_status hplmm_sg_get_grads(const hplmm_sg_net *net, float *host, int64_t count, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the last gradients. */
hplmm_status hplmm_sg_adam(hplmm_sg_net *net, float lr, void *stream);

void hplmm_sg_destroy(hplmm_sg_net *net);

/* Samples of a planned problem: one per (grain, adjacent interface c, mortar
 * a), ordered by grain, then interface id, then a.  Writes the network inputs
 * of samples first .. first + count - 1 to x_dev[count][729][4] and, if y_dev
 * is not NULL, their exact targets (the grain's shape vectors of columns
 * 3a + x, y, z after hplmm_setup) to y_dev[count][729][9]; meta (host, may be NULL) receives
 * {grain matrix index, interface id, mortar index} per sample.  *total (may
 * be NULL) receives the number of samples; count = 0 only queries it.
 * Grains must be 8^3-voxel boxes (every grain node and every node of its
 * adjacent interfaces inside one 9^3 node lattice with a corner at a multiple
 * of 8): E_PARTITION otherwise; the mortars must be Gaussian: E_ARG otherwise.  E_STATE if targets are asked before setup.
 * Asynchronous on stream except the first call, which builds and uploads the
 * sample tables. */
hplmm_status hplmm_sg_samples(hplmm_handle *h, int64_t first, int64_t count, float *x_dev, float *y_dev,
                              int32_t *meta, int64_t *total, void *stream);

/* Set-up with learned shape vectors (Eq. 23).  Same as hplmm_setup, except
 * that the network predicts the shape vectors of every grain; a grain keeps
 * them when it has no correction column and every mortar column k passes the
 * local residual check |A_gi p~_k + Abar_gi,m e_k| <= threshold
 * |Abar_gi,m e_k| (residuals from the grain's Cholesky factor); every other
 * grain gets the exact shape vectors.  The coarse operator is the Galerkin
 * product with the resulting basis on the mortar block (Eq. 18) plus the exact
 * correction pivots; the mortar-correction coupling, zero for exact shape
 * vectors, is not formed.  threshold = 0 reproduces hplmm_setup's basis.
 * net must map 4 input channels to 9 outputs.  stats (may be NULL) receives
 * counts, the residual ratios and host-clock phase times. */
typedef struct hplmm_sg_stats {
    int32_t grains;                 /* grain matrices */
    int32_t accepted;               /* grains that kept the predicted shape vectors */
    int32_t fallback;               /* grains given the exact shape vectors */
    int32_t loaded;                 /* grains with a correction column (always exact) */
    double  max_residual_accepted;  /* largest residual ratio among accepted columns */
    double  median_residual;        /* median residual ratio over all predicted columns */
    double  t_infer_ms;             /* inference (synchronised) */
    double  t_check_ms;             /* residual check */
    double  t_basis_ms;             /* exact fallback and Galerkin blocks */
} hplmm_sg_stats;

hplmm_status hplmm_setup_surrogate(hplmm_handle *h, hplmm_sg_net *net, double threshold, hplmm_sg_stats *stats,
                                   void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HPLMM_SURROGATE_H */
