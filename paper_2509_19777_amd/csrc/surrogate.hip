// Convolution kernels of the learned basis surrogate on the matrix cores.
//
// A 3x3x3 'same' convolution on the 9^3 lattice is an implicit GEMM: rows =
// lattice positions, columns = output channels, and the contraction runs over
// the 27 kernel offsets times the input channels.  A work-group owns 64
// positions of one sample; for each offset it gathers the 64 shifted input
// rows and that offset's weight slice into LDS and multiplies them with
// v_mfma_f32_16x16x4f32 (four wavefronts, 16 positions each).  The data
// gradient is the same product with reversed offsets and transposed weight
// slices; the weight gradient contracts over positions instead.
#include <hip/hip_runtime.h>

#include "surrogate.h"

namespace hplmm {
namespace sg {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// lattice neighbour of position p at offset index d, or -1 outside
__device__ __forceinline__ int neighbour(int p, int d) {
    const int x = p % G, y = (p / G) % G, z = p / (G * G);
    const int xx = x + d % 3 - 1, yy = y + (d / 3) % 3 - 1, zz = z + d / 9 - 1;
    if (xx < 0 || yy < 0 || zz < 0 || xx >= G || yy >= G || zz >= G) return -1;
    return (zz * G + yy) * G + xx;
}

// KIN: input channels padded to a multiple of 4; NOUT: output channels padded
// to a multiple of 16.  BWD: data gradient (offsets reversed, weights read as
// w[26 - d][n][k]).
template <int KIN, int NOUT, bool BWD>
__global__ void __launch_bounds__(256) conv_kernel(const float *__restrict__ in, int cin, const float *__restrict__ w,
                                                   int wc0, int wc1, const float *__restrict__ bias,
                                                   const float *__restrict__ mask, float *__restrict__ out, int cout,
                                                   int relu) {
    __shared__ float Xs[64][KIN + 1];
    __shared__ float Ws[KIN][NOUT + 1];
    const int s = blockIdx.y;
    const int p0 = blockIdx.x * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    v4f acc[NOUT / 16];
#pragma unroll
    for (int nb = 0; nb < NOUT / 16; ++nb) acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
    const float *ins = in + (int64_t)s * P * cin;
    for (int d = 0; d < NOFF; ++d) {
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * KIN; e += 256) {
            const int pl = e / KIN, k = e % KIN;
            const int p = p0 + pl;
            float v = 0.f;
            if (p < P && k < cin) {
                const int q = neighbour(p, d);
                if (q >= 0) v = ins[q * cin + k];
            }
            Xs[pl][k] = v;
        }
        for (int e = threadIdx.x; e < KIN * NOUT; e += 256) {
            const int k = e / NOUT, n = e % NOUT;
            float v = 0.f;
            if (!BWD) {
                if (k < wc0 && n < wc1) v = w[((int64_t)d * wc0 + k) * wc1 + n];
            } else {
                if (n < wc0 && k < wc1) v = w[((int64_t)(NOFF - 1 - d) * wc0 + n) * wc1 + k];
            }
            Ws[k][n] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KIN / 4; ++kk) {
            const float a = Xs[16 * wave + lr][4 * kk + lk];
#pragma unroll
            for (int nb = 0; nb < NOUT / 16; ++nb) acc[nb] = mfma(a, Ws[4 * kk + lk][16 * nb + lr], acc[nb]);
        }
    }
    float *outs = out + (int64_t)s * P * cout;
#pragma unroll
    for (int nb = 0; nb < NOUT / 16; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = p0 + 16 * wave + 4 * lk + r;
            const int n = 16 * nb + lr;
            if (p >= P || n >= cout) continue;
            float v = acc[nb][r];
            if (bias) v += bias[n];
            if (relu) v = v > 0.f ? v : 0.f;
            if (mask && !(mask[((int64_t)s * P + p) * cout + n] > 0.f)) v = 0.f;
            outs[p * cout + n] = v;
        }
}

// Forward convolution with bfloat16 operands (inference): the staged input
// rows and weight slices are rounded to bfloat16 (to nearest even) and one
// v_mfma_f32_16x16x32_bf16 per 16 output channels contracts all 32 (padded)
// input channels of an offset, with FP32 accumulation; bias, ReLU and the
// stored activations stay FP32.  Lane l supplies position (or output channel)
// l & 15 at channels 8 (l >> 4) .. + 7, one 16-byte LDS read each.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
constexpr int KB = 32, KBL = KB + 8;   // channels per offset, padded LDS row (bf16 elements)

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int NOUT>
__global__ void __launch_bounds__(256) conv_fwd_bf16_kernel(const float *__restrict__ in, int cin,
                                                            const float *__restrict__ w,
                                                            const float *__restrict__ bias, float *__restrict__ out,
                                                            int cout, int relu) {
    __shared__ __align__(16) uint16_t Xs[64][KBL];
    __shared__ __align__(16) uint16_t Ws[NOUT][KBL];   // w^T: [co][ci]
    const int s = blockIdx.y;
    const int p0 = blockIdx.x * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, k0 = 8 * (lane >> 4);
    v4f acc[NOUT / 16];
#pragma unroll
    for (int nb = 0; nb < NOUT / 16; ++nb) acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
    const float *ins = in + (int64_t)s * P * cin;
    for (int d = 0; d < NOFF; ++d) {
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * KB; e += 256) {
            const int pl = e / KB, k = e % KB;
            const int p = p0 + pl;
            float v = 0.f;
            if (p < P && k < cin) {
                const int q = neighbour(p, d);
                if (q >= 0) v = ins[q * cin + k];
            }
            Xs[pl][k] = to_bf16(v);
        }
        for (int e = threadIdx.x; e < KB * NOUT; e += 256) {
            const int k = e / NOUT, n = e % NOUT;
            Ws[n][k] = to_bf16((k < cin && n < cout) ? w[((int64_t)d * cin + k) * cout + n] : 0.f);
        }
        __syncthreads();
        const v8bf a = *reinterpret_cast<const v8bf *>(&Xs[16 * wave + lr][k0]);
#pragma unroll
        for (int nb = 0; nb < NOUT / 16; ++nb) {
            const v8bf b = *reinterpret_cast<const v8bf *>(&Ws[16 * nb + lr][k0]);
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[nb], 0, 0, 0);
        }
    }
    float *outs = out + (int64_t)s * P * cout;
#pragma unroll
    for (int nb = 0; nb < NOUT / 16; ++nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = p0 + 16 * wave + 4 * (lane >> 4) + r;
            const int n = 16 * nb + lr;
            if (p >= P || n >= cout) continue;
            float v = acc[nb][r];
            if (bias) v += bias[n];
            if (relu) v = v > 0.f ? v : 0.f;
            outs[p * cout + n] = v;
        }
}

void launch_conv_fwd_bf16(const float *in, int cin, const float *w, const float *bias, float *out, int cout, int n,
                          int relu, hipStream_t s) {
    if (n <= 0) return;
    const dim3 grid((P + 63) / 64, n);
    if (cout <= 16)
        hipLaunchKernelGGL(conv_fwd_bf16_kernel<16>, grid, dim3(256), 0, s, in, cin, w, bias, out, cout, relu);
    else
        hipLaunchKernelGGL(conv_fwd_bf16_kernel<32>, grid, dim3(256), 0, s, in, cin, w, bias, out, cout, relu);
}

template <bool BWD>
static void conv_dispatch(const float *in, int cin, const float *w, int wc0, int wc1, const float *bias,
                          const float *mask, float *out, int cout, int n, int relu, hipStream_t s) {
    if (n <= 0) return;
    const dim3 grid((P + 63) / 64, n);
    const int kin = cin <= 4 ? 4 : (cin <= 16 ? 16 : 32);
    const int nout = cout <= 16 ? 16 : 32;
#define SG_CONV(K, N)                                                                                              \
    hipLaunchKernelGGL((conv_kernel<K, N, BWD>), grid, dim3(256), 0, s, in, cin, w, wc0, wc1, bias, mask, out, cout, \
                       relu)
    if (kin == 4 && nout == 16) SG_CONV(4, 16);
    else if (kin == 4) SG_CONV(4, 32);
    else if (kin == 16 && nout == 16) SG_CONV(16, 16);
    else if (kin == 16) SG_CONV(16, 32);
    else if (nout == 16) SG_CONV(32, 16);
    else SG_CONV(32, 32);
#undef SG_CONV
}

void launch_conv_fwd(const float *in, int cin, const float *w, const float *bias, float *out, int cout, int n,
                     int relu, hipStream_t s) {
    conv_dispatch<false>(in, cin, w, cin, cout, bias, nullptr, out, cout, n, relu, s);
}

void launch_conv_bwd_data(const float *g, int cout, const float *w, float *gin, int cin, const float *act, int n,
                          hipStream_t s) {
    // the "input" is g (cout channels), the "output" gin (cin channels); the
    // weight is still stored as w[d][ci][co] = (wc0 = cin, wc1 = cout)
    conv_dispatch<true>(g, cout, w, cin, cout, nullptr, act, gin, cin, n, 0, s);
}

// Weight gradient: work-group (offset d, chunk c) contracts over the positions
// of samples c, c + chunks, ...; wave (mb, nb) owns a 16x16 block of (ci, co).
template <int KIN, int NOUT>
__global__ void __launch_bounds__(256) conv_wgrad_kernel(const float *__restrict__ in, int cin,
                                                         const float *__restrict__ g, int cout, int n, int chunks,
                                                         float *__restrict__ part) {
    __shared__ float Xs[64][KIN + 1];
    __shared__ float Gs[64][NOUT + 1];
    const int d = blockIdx.x, c = blockIdx.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    constexpr int MB = (KIN + 15) / 16, NB = NOUT / 16;
    const int mb = wave % MB, nb = wave / MB;
    const bool active = wave < MB * NB;
    v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
    for (int s = c; s < n; s += chunks) {
        const float *ins = in + (int64_t)s * P * cin;
        const float *gs = g + (int64_t)s * P * cout;
        for (int p0 = 0; p0 < P; p0 += 64) {
            __syncthreads();
            for (int e = threadIdx.x; e < 64 * KIN; e += 256) {
                const int pl = e / KIN, k = e % KIN;
                const int p = p0 + pl;
                float v = 0.f;
                if (p < P && k < cin) {
                    const int q = neighbour(p, d);
                    if (q >= 0) v = ins[q * cin + k];
                }
                Xs[pl][k] = v;
            }
            for (int e = threadIdx.x; e < 64 * NOUT; e += 256) {
                const int pl = e / NOUT, k = e % NOUT;
                const int p = p0 + pl;
                Gs[pl][k] = (p < P && k < cout) ? gs[p * cout + k] : 0.f;
            }
            __syncthreads();
            if (active) {
#pragma unroll
                for (int kk = 0; kk < 16; ++kk) {
                    const int m = 16 * mb + lr;
                    const float a = m < KIN ? Xs[4 * kk + lk][m] : 0.f;
                    acc = mfma(a, Gs[4 * kk + lk][16 * nb + lr], acc);
                }
            }
        }
    }
    if (!active) return;
    float *pc = part + (int64_t)c * (NOFF * cin * cout + cout) + (int64_t)d * cin * cout;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int m = 16 * mb + 4 * lk + r, nn = 16 * nb + lr;
        if (m < cin && nn < cout) pc[m * cout + nn] = acc[r];
    }
}

// bias partials: part[c][27 cin cout + co] = sum over the chunk's samples and positions
__global__ void __launch_bounds__(256) conv_bgrad_kernel(const float *__restrict__ g, int cin, int cout, int n,
                                                         int chunks, float *__restrict__ part) {
    __shared__ float red[256];
    const int c = blockIdx.x;
    for (int co = 0; co < cout; ++co) {
        float t = 0.f;
        for (int s = c; s < n; s += chunks)
            for (int p = threadIdx.x; p < P; p += 256) t += g[((int64_t)s * P + p) * cout + co];
        red[threadIdx.x] = t;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)c * (NOFF * cin * cout + cout) + NOFF * cin * cout + co] = red[0];
        __syncthreads();
    }
}

__global__ void reduce_chunks_kernel(const float *__restrict__ part, int chunks, int64_t len,
                                     float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    float t = 0.f;
    for (int c = 0; c < chunks; ++c) t += part[(int64_t)c * len + i];
    out[i] = t;
}

void launch_conv_bwd_weight(const float *in, int cin, const float *g, int cout, int n, float *part, int chunks,
                            float *gwb, hipStream_t s) {
    if (n <= 0) return;
    const int kin = cin <= 4 ? 4 : (cin <= 16 ? 16 : 32);
    const int nout = cout <= 16 ? 16 : 32;
    const dim3 grid(NOFF, chunks);
#define SG_WG(K, N) hipLaunchKernelGGL((conv_wgrad_kernel<K, N>), grid, dim3(256), 0, s, in, cin, g, cout, n, chunks, part)
    if (kin == 4 && nout == 16) SG_WG(4, 16);
    else if (kin == 4) SG_WG(4, 32);
    else if (kin == 16 && nout == 16) SG_WG(16, 16);
    else if (kin == 16) SG_WG(16, 32);
    else if (nout == 16) SG_WG(32, 16);
    else SG_WG(32, 32);
#undef SG_WG
    hipLaunchKernelGGL(conv_bgrad_kernel, dim3(chunks), dim3(256), 0, s, g, cin, cout, n, chunks, part);
    const int64_t len = (int64_t)NOFF * cin * cout + cout;
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, part, chunks, len,
                       gwb);
}

// One work-group per sample: the masked norms by a fixed-order tree, then the gradient.
__global__ void __launch_bounds__(256) loss_kernel(const float *__restrict__ pred, const float *__restrict__ y,
                                                   int c, const float *__restrict__ x, int cx, int n,
                                                   float *__restrict__ gpred, double *__restrict__ loss_s) {
    __shared__ double rn[256], rd[256];
    const int s = blockIdx.x;
    double num = 0.0, den = 0.0;
    for (int e = threadIdx.x; e < P * c; e += 256) {
        const int p = e / c;
        if (!(x[((int64_t)s * P + p) * cx] > 0.5f)) continue;
        const double yv = y[(int64_t)s * P * c + e], dv = (double)pred[(int64_t)s * P * c + e] - yv;
        num += dv * dv;
        den += yv * yv;
    }
    rn[threadIdx.x] = num;
    rd[threadIdx.x] = den;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            rn[threadIdx.x] += rn[threadIdx.x + w];
            rd[threadIdx.x] += rd[threadIdx.x + w];
        }
        __syncthreads();
    }
    const double dd = rd[0] + 1e-30;
    if (threadIdx.x == 0) loss_s[s] = rn[0] / dd;
    const double scale = 2.0 / (dd * n);
    for (int e = threadIdx.x; e < P * c; e += 256) {
        const int p = e / c;
        const int64_t i = (int64_t)s * P * c + e;
        gpred[i] = (x[((int64_t)s * P + p) * cx] > 0.5f) ? (float)(scale * ((double)pred[i] - (double)y[i])) : 0.f;
    }
}

void launch_loss(const float *pred, const float *y, int c, const float *x, int cx, int n, float *gpred,
                 double *loss_s, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(loss_kernel, dim3(n), dim3(256), 0, s, pred, y, c, x, cx, n, gpred, loss_s);
}

__global__ void adam_kernel(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

void launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
                 float eps, int t, hipStream_t s) {
    if (n <= 0) return;
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr, beta1,
                       beta2, eps, c1, c2);
}

// ---- samples of a set-up problem ---------------------------------------------------
__device__ __forceinline__ int lattice_pos(const SampleArgs &a, int32_t v, int m) {
    const int x = a.xyz[3 * (int64_t)v] - a.g_origin[3 * m];
    const int y = a.xyz[3 * (int64_t)v + 1] - a.g_origin[3 * m + 1];
    const int z = a.xyz[3 * (int64_t)v + 2] - a.g_origin[3 * m + 2];
    return (z * G + y) * G + x;   // the host checked 0 <= x, y, z < G
}

__global__ void __launch_bounds__(256) fill_samples_kernel(SampleArgs a, int64_t first, float *__restrict__ x,
                                                           float *__restrict__ y) {
    const int64_t sl = blockIdx.x, s = first + sl;
    const int m = a.s_m[s], c = a.s_c[s], am = a.s_a[s], lcol = a.s_lcol[s];
    float *xs = x + sl * P * 4;
    for (int e = threadIdx.x; e < P * 4; e += 256) xs[e] = 0.f;
    float *ys = y ? y + sl * P * 9 : nullptr;
    if (ys)
        for (int e = threadIdx.x; e < P * 9; e += 256) ys[e] = 0.f;
    __syncthreads();
    // fill channel of every adjacent interface's nodes
    for (int64_t q = a.adj_ptr[m]; q < a.adj_ptr[m + 1]; ++q) {
        const int ci = a.adj[q];
        for (int64_t t = a.iface_ptr[ci] + threadIdx.x; t < a.iface_ptr[ci + 1]; t += 256) {
            const int32_t v = a.iface_nodes[t];
            xs[lattice_pos(a, v, m) * 4 + 2] = a.fill[v];
        }
    }
    // boundary trace of mortar am of interface c
    {
        const int nu = a.iface_nu[c];
        const int64_t p0 = a.iface_ptr[c];
        for (int64_t t = p0 + threadIdx.x; t < a.iface_ptr[c + 1]; t += 256) {
            const int32_t v = a.iface_nodes[t];
            xs[lattice_pos(a, v, m) * 4 + 3] = (float)a.H[a.iface_hoff[c] + (t - p0) * nu + am];
        }
    }
    // interior nodes: indicator, log-trace, fill; targets
    const int64_t nd = a.g_ndof[m], vo = a.g_voff[m], ro = a.g_roff[m], nt = a.g_nt[m];
    for (int64_t i = threadIdx.x; i < nd; i += 256) {
        const int64_t dof = a.slot_dof[vo + i];
        const int32_t v = (int32_t)(dof / 3);
        const int comp = (int)(dof - 3 * (int64_t)v);
        const int p = lattice_pos(a, v, m);
        if (comp == 0) {
            xs[p * 4 + 0] = 1.f;
            xs[p * 4 + 1] = a.logtr[v] - a.g_logmean[m];
            xs[p * 4 + 2] = a.fill[v];
        }
        if (ys)
            for (int gm = 0; gm < 3; ++gm) {
                const int64_t j = lcol + 3 * am + gm;
                const double val = a.X[ro + ((j / 64) * nt + i / 64) * 4096 + (i % 64) + 64 * (j % 64)];
                ys[p * 9 + 3 * gm + comp] = (float)val;
            }
    }
}

void launch_fill_samples(const SampleArgs &a, int64_t first, int64_t count, float *x, float *y, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(fill_samples_kernel, dim3((unsigned)count), dim3(256), 0, s, a, first, x, y);
}

__global__ void __launch_bounds__(256) scatter_pred_kernel(SampleArgs a, int64_t first, const float *__restrict__ y,
                                                           double *__restrict__ arena) {
    const int64_t sl = blockIdx.x, s = first + sl;
    const int m = a.s_m[s], am = a.s_a[s], lcol = a.s_lcol[s];
    const float *ys = y + sl * P * 9;
    const int64_t nd = a.g_ndof[m], vo = a.g_voff[m], ro = a.g_roff[m], nt = a.g_nt[m];
    for (int64_t i = threadIdx.x; i < nd; i += 256) {
        const int64_t dof = a.slot_dof[vo + i];
        const int32_t v = (int32_t)(dof / 3);
        const int comp = (int)(dof - 3 * (int64_t)v);
        const int p = lattice_pos(a, v, m);
        for (int gm = 0; gm < 3; ++gm) {
            const int64_t j = lcol + 3 * am + gm;
            arena[ro + ((j / 64) * nt + i / 64) * 4096 + (i % 64) + 64 * (j % 64)] = (double)ys[p * 9 + 3 * gm + comp];
        }
    }
}

void launch_scatter_pred(const SampleArgs &a, int64_t first, int64_t count, const float *y, double *arena,
                         hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(scatter_pred_kernel, dim3((unsigned)count), dim3(256), 0, s, a, first, y, arena);
}

// one work-group per (block, column tile): 64 columns x 4 row groups, fixed-order sums
__global__ void __launch_bounds__(256) col_norms_kernel(const double *__restrict__ arena, const int64_t *__restrict__ off,
                                                        const int32_t *__restrict__ nt, const int32_t *__restrict__ ctile,
                                                        const int64_t *__restrict__ cofs,
                                                        const int32_t *__restrict__ ncol, double *__restrict__ out) {
    __shared__ double red[4][64];
    const int t = blockIdx.x;
    const int j = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const int64_t base = off[t] + (int64_t)ctile[t] * nt[t] * 4096;
    double acc = 0.0;
    for (int I = 0; I < nt[t]; ++I)
        for (int r = rg; r < 64; r += 4) {
            const double v = arena[base + (int64_t)I * 4096 + j * 64 + r];
            acc += v * v;
        }
    red[rg][j] = acc;
    __syncthreads();
    if (rg == 0) {
        const int col = ctile[t] * 64 + j;
        if (col < ncol[t]) out[cofs[t] + col] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
    }
}

void launch_col_norms(const double *arena, const int64_t *off, const int32_t *nt, const int32_t *ctile,
                      const int64_t *cofs, const int32_t *ncol, int64_t ntasks, double *out, hipStream_t s) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(col_norms_kernel, dim3((unsigned)ntasks), dim3(256), 0, s, arena, off, nt, ctile, cofs, ncol,
                       out);
}

}  // namespace sg
}  // namespace hplmm
