// Kernels of the learned basis surrogate: a 3D convolutional network on the
// 9 x 9 x 9 node lattice of a box subdomain (four 3x3x3 'same' convolutions
// with bias, ReLU after the first three), its training (loss, gradients, Adam)
// and its inference.  Activations are float32, channel-last:
// act[s][p][c] with p = (z * 9 + y) * 9 + x.  Weights w[d][ci][co] with
// d = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1), then the biases b[co].
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hplmm {
namespace sg {

constexpr int G = 9;
constexpr int P = G * G * G;
constexpr int NOFF = 27;

// out[s][p][co] = bias[co] + sum_{d, ci} w[d][ci][co] in[s][p + o(d)][ci]
// (zero outside the lattice), then ReLU when relu != 0.  cin <= 32, cout <= 32.
void launch_conv_fwd(const float *in, int cin, const float *w, const float *bias, float *out, int cout, int n,
                     int relu, hipStream_t s);
// The same with the staged inputs and weights rounded to bfloat16 (to
// nearest even), FP32 accumulation and FP32 output (inference).
void launch_conv_fwd_bf16(const float *in, int cin, const float *w, const float *bias, float *out, int cout, int n,
                          int relu, hipStream_t s);
// gin[s][p][ci] = [act[s][p][ci] > 0] sum_{d, co} w[d][ci][co] g[s][p - o(d)][co]
// (act may be null: no mask).  g has cout channels, gin cin.
void launch_conv_bwd_data(const float *g, int cout, const float *w, float *gin, int cin, const float *act, int n,
                          hipStream_t s);
// gw[d][ci][co] = sum_{s, p} in[s][p + o(d)][ci] g[s][p][co] and gb[co] = sum_{s, p} g[s][p][co]:
// per-chunk partials in part (chunks * (27 cin cout + cout) floats), then a
// fixed-order reduction into gw (27 cin cout floats) followed by gb.
void launch_conv_bwd_weight(const float *in, int cin, const float *g, int cout, int n, float *part, int chunks,
                            float *gwb, hipStream_t s);
// Per-sample loss |m (pred - y)|^2 / (|m y|^2 + 1e-30) over the first c
// channels, m = [x[s][p][0] > 0.5] (x has cx channels); gpred = d mean / d pred;
// loss_s[s] receives each sample's term.
void launch_loss(const float *pred, const float *y, int c, const float *x, int cx, int n, float *gpred,
                 double *loss_s, hipStream_t s);
// Adam with bias correction at step t (>= 1).
void launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
                 float eps, int t, hipStream_t s);

// Index data of the (grain, interface, mortar) samples of a set-up problem.
struct SampleArgs {
    const int32_t *s_m, *s_c, *s_a, *s_lcol;   // per sample: grain matrix, interface, mortar, first column
    const int32_t *g_origin;                   // [3 nG] lattice coordinates of each grain's box corner
    const int64_t *g_voff, *g_ndof, *g_roff, *g_nt;
    const float *g_logmean;                    // [nG] mean log trace over the grain's interior nodes
    const int64_t *adj_ptr;                    // grain -> adjacent interfaces
    const int32_t *adj;
    const int64_t *iface_ptr;                  // interface -> nodes
    const int32_t *iface_nodes;
    const double *H;                           // Gaussian weights, per interface row-major N_c x nu_c
    const int64_t *iface_hoff;
    const int32_t *iface_nu;
    const int32_t *xyz;                        // [3 n_nodes]
    const float *logtr, *fill;                 // [n_nodes]
    const int64_t *slot_dof;                   // grain vector slot -> dof
    const double *X;                           // arena holding each grain's shape vectors B = -A_gi^-1 Abar_gi (tiles)
};
// x[s][p][4] inputs and, when y is not null, y[s][p][9] targets (columns
// lcol + 3a + gamma of B at the interior nodes) for samples first .. first + count.
void launch_fill_samples(const SampleArgs &a, int64_t first, int64_t count, float *x, float *y, hipStream_t s);
// The inverse map for predictions: column lcol + 3a + gamma of the grain's
// shape-vector block (tile grid at g_roff of the arena) receives
// y[s][p][3 gamma + comp] at its interior rows, for samples first .. first + count.
void launch_scatter_pred(const SampleArgs &a, int64_t first, int64_t count, const float *y, double *arena,
                         hipStream_t s);
// Squared column norms of tile-grid blocks: task t covers grain block
// (arena offset off[t], nt[t] row tiles) column tile ctile[t]; column j of the
// block lands at out[cofs[t] + j] for j < ncol[t].
void launch_col_norms(const double *arena, const int64_t *off, const int32_t *nt, const int32_t *ctile,
                      const int64_t *cofs, const int32_t *ncol, int64_t ntasks, double *out, hipStream_t s);

}  // namespace sg
}  // namespace hplmm
