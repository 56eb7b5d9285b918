// Sparse, gather/scatter, coarse-assembly and Krylov kernels for gfx950.
//
// Every kernel writes each output element from exactly one thread and sums
// in a fixed order, so results are bitwise reproducible run to run (no
// floating-point atomics).
#include <hip/hip_runtime.h>

#include "dense.h"
#include "sparse.h"

#include <algorithm>

namespace hplmm {

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// ---- SpMV (SELL-64, one wavefront per slice, one lane per node row) ---------
__global__ void __launch_bounds__(256) spmv_kernel(int64_t n_rows, int32_t n_slices,
                                                   const int64_t *__restrict__ slice_step,
                                                   const int32_t *__restrict__ col,
                                                   const double *__restrict__ val,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ r, double *__restrict__ y) {
    const int lane = threadIdx.x & 63;
    const int slice = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (slice >= n_slices) return;
    const int64_t st = slice_step[slice], en = slice_step[slice + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t k = st; k < en; ++k) {
        const int64_t c = col[k * SELL_C + lane];
        const double *v = val + k * (9 * SELL_C) + lane;
        const double x0 = x[3 * c], x1 = x[3 * c + 1], x2 = x[3 * c + 2];
        a0 += v[0] * x0 + v[64] * x1 + v[128] * x2;
        a1 += v[192] * x0 + v[256] * x1 + v[320] * x2;
        a2 += v[384] * x0 + v[448] * x1 + v[512] * x2;
    }
    const int64_t row = (int64_t)slice * SELL_C + lane;
    if (row < n_rows) {
        if (r) {
            y[3 * row] = r[3 * row] - a0;
            y[3 * row + 1] = r[3 * row + 1] - a1;
            y[3 * row + 2] = r[3 * row + 2] - a2;
        } else {
            y[3 * row] = a0;
            y[3 * row + 1] = a1;
            y[3 * row + 2] = a2;
        }
    }
}

void launch_spmv(const SellMatrix &A, const double *x, const double *r, double *y, hipStream_t s) {
    hipLaunchKernelGGL(spmv_kernel, dim3(blocks_for(A.n_slices, 4)), dim3(256), 0, s, A.n_rows, A.n_slices,
                       A.slice_step, A.col, A.val, x, r, y);
}

// ---- gathers / combination ----------------------------------------------------
__global__ void gather_kernel(const int64_t *__restrict__ map, const double *__restrict__ src,
                              double *__restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t m = map[i];
    dst[i] = m >= 0 ? src[m] : 0.0;
}
void launch_gather(const int64_t *map, const double *src, double *dst, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(gather_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, map, src, dst, n);
}

__global__ void combine_kernel(int64_t n, const double *__restrict__ base, const int64_t *__restrict__ gslot,
                               const double *__restrict__ g, const int64_t *__restrict__ cptr,
                               const int64_t *__restrict__ cslot, const double *__restrict__ c,
                               double *__restrict__ out) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= n) return;
    double s = base ? base[d] : 0.0;
    if (gslot) {
        const int64_t q = gslot[d];
        if (q >= 0) s += g[q];
    }
    if (cptr) {
        double t = 0.0;
        for (int64_t p = cptr[d]; p < cptr[d + 1]; ++p) t += c[cslot[p]];
        s += t;
    }
    out[d] = s;
}
void launch_combine(int64_t n, const double *base, const int64_t *gslot, const double *g, const int64_t *cptr,
                    const int64_t *cslot, const double *c, double *out, hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, base, gslot, g, cptr, cslot,
                       c, out);
}

// ---- restriction / prolongation ------------------------------------------------
// One coarse dof's sum, by one wavefront: the lanes share the interface's
// node sum and the per-grain restriction terms, then a fixed butterfly adds
// them up (every lane ends with the total).
__device__ __forceinline__ double coarse_rhs_dof(const CoarseMaps &m, int64_t q, const double *__restrict__ r,
                                                 const double *__restrict__ t, int lane) {
    double s = 0.0;
    if (q < m.n_mortar) {
        const int32_t c = m.q_iface[q];
        const int32_t lq = m.q_local[q];
        const int32_t nu = m.iface_nu[c];
        const int32_t a = lq / 3, d = lq % 3;
        const double *H = m.H + m.iface_hoff[c];
        const int64_t p0 = m.iface_ptr[c], p1 = m.iface_ptr[c + 1];
        if (!m.general) {
            for (int64_t p = p0 + lane; p < p1; p += 64) s += H[(p - p0) * nu + a] * r[3 * (int64_t)m.iface_nodes[p] + d];
        } else {
            const int64_t k3 = 3 * (int64_t)nu;
            for (int64_t p = p0 + lane; p < p1; p += 64) {
                const double *row = H + 3 * (p - p0) * k3 + lq;
                const double *rv = r + 3 * (int64_t)m.iface_nodes[p];
                s += row[0] * rv[0] + row[k3] * rv[1] + row[2 * k3] * rv[2];
            }
        }
    }
    for (int64_t p = m.tptr[q] + lane; p < m.tptr[q + 1]; p += 64) s += t[m.tslot[p]];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// With Gaussian mortars one wavefront takes a whole interface: it reads the
// node values and the rows of H once, accumulating all 3 nu sums together,
// adds each up with the same butterfly, and lane j = 3 a + d finishes mortar
// dof moff + j with its per-grain terms.  Interfaces of more than RHS_MAXNU
// functions, the general blocks and the corrections go one dof per wavefront.
constexpr int RHS_MAXNU = 4;
__global__ void __launch_bounds__(256) coarse_rhs_kernel(CoarseMaps m, const double *__restrict__ r,
                                                         const double *__restrict__ t, double *__restrict__ f) {
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t nw_if = m.general ? 0 : m.n_ifaces;
    if (w < nw_if) {
        const int32_t c = (int32_t)w;
        const int32_t nu = m.iface_nu[c];
        const int64_t mo = m.iface_moff[c];
        if (nu > RHS_MAXNU) {
            for (int j = 0; j < 3 * nu; ++j) {
                const double s = coarse_rhs_dof(m, mo + j, r, t, lane);
                if (lane == 0) f[m.fpos[mo + j]] = s;
            }
            return;
        }
        double acc[RHS_MAXNU][3];
#pragma unroll
        for (int a = 0; a < RHS_MAXNU; ++a) acc[a][0] = acc[a][1] = acc[a][2] = 0.0;
        const double *H = m.H + m.iface_hoff[c];
        const int64_t p0 = m.iface_ptr[c], p1 = m.iface_ptr[c + 1];
        for (int64_t p = p0 + lane; p < p1; p += 64) {
            const double *rv = r + 3 * (int64_t)m.iface_nodes[p];
            const double r0 = rv[0], r1 = rv[1], r2 = rv[2];
            const double *hp = H + (p - p0) * nu;
#pragma unroll
            for (int a = 0; a < RHS_MAXNU; ++a)
                if (a < nu) {
                    const double ha = hp[a];
                    acc[a][0] += ha * r0;
                    acc[a][1] += ha * r1;
                    acc[a][2] += ha * r2;
                }
        }
        double mine = 0.0;
#pragma unroll
        for (int a = 0; a < RHS_MAXNU; ++a)
            if (a < nu) {   // nu is the same across the wavefront
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    double v = acc[a][d];
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
                    if (lane == 3 * a + d) mine = v;
                }
            }
        if (lane < 3 * nu) {
            const int64_t q = mo + lane;
            for (int64_t p = m.tptr[q]; p < m.tptr[q + 1]; ++p) mine += t[m.tslot[p]];
            f[m.fpos[q]] = mine;
        }
        return;
    }
    const int64_t q = m.general ? w : m.n_mortar + (w - nw_if);
    if (q >= m.n_coarse) return;
    const double s = coarse_rhs_dof(m, q, r, t, lane);
    if (lane == 0) f[m.fpos[q]] = s;
}
void launch_coarse_rhs(const CoarseMaps &m, const double *r, const double *t, double *f, hipStream_t s) {
    if (m.n_coarse <= 0) return;
    const int64_t waves = m.general ? m.n_coarse : m.n_ifaces + (m.n_coarse - m.n_mortar);
    if (waves <= 0) return;
    hipLaunchKernelGGL(coarse_rhs_kernel, dim3(blocks_for(waves, 4)), dim3(256), 0, s, m, r, t, f);
}

__global__ void corr_solve_kernel(CoarseMaps m, const double *__restrict__ f, double *__restrict__ u) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t q = m.n_mortar + j;
    if (q >= m.n_coarse) return;
    u[m.fpos[q]] = f[m.fpos[q]] / m.corr_d[j];
}
void launch_corr_solve(const CoarseMaps &m, const double *f, double *u, hipStream_t s) {
    const int64_t nc = m.n_coarse - m.n_mortar;
    if (nc <= 0) return;
    hipLaunchKernelGGL(corr_solve_kernel, dim3(blocks_for(nc, 256)), dim3(256), 0, s, m, f, u);
}

__global__ void prolong_nodes_kernel(CoarseMaps m, int64_t n_nodes, const int64_t *__restrict__ gslot,
                                     const double *__restrict__ zl, const double *__restrict__ u,
                                     double *__restrict__ z) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= 3 * n_nodes) return;
    const int64_t q = gslot[d];
    if (q >= 0) {
        z[d] = zl[q];
        return;
    }
    const int64_t v = d / 3;
    const int g = (int)(d - 3 * v);
    const int32_t c = m.node_iface[v];
    double s = 0.0;
    if (c >= 0) {
        const int32_t nu = m.iface_nu[c];
        const int64_t mo = m.iface_moff[c];
        if (!m.general) {
            const double *H = m.H + m.iface_hoff[c] + (int64_t)m.node_irow[v] * nu;
            for (int a = 0; a < nu; ++a) s += H[a] * u[m.fpos[mo + 3 * a + g]];
        } else {
            const int64_t k3 = 3 * (int64_t)nu;
            const double *H = m.H + m.iface_hoff[c] + (3 * (int64_t)m.node_irow[v] + g) * k3;
            for (int64_t k = 0; k < k3; ++k) s += H[k] * u[m.fpos[mo + k]];
        }
    }
    z[d] = s;
}
void launch_prolong_nodes(const CoarseMaps &m, int64_t n_nodes, const int64_t *gslot, const double *zl,
                          const double *u, double *z, hipStream_t s) {
    hipLaunchKernelGGL(prolong_nodes_kernel, dim3(blocks_for(3 * n_nodes, 256)), dim3(256), 0, s, m, n_nodes,
                       gslot, zl, u, z);
}

// ---- set-up gathers ------------------------------------------------------------
__device__ __forceinline__ int64_t tile_elem(int64_t r, int64_t c) {
    // element (r, c) inside packed lower tiles (caller ensures r/64 >= c/64)
    const int64_t I = r >> 6, J = c >> 6;
    return tri_index(I, J) * TE + (c & 63) * TS + (r & 63);
}
__device__ __forceinline__ int64_t rect_elem(int64_t r, int64_t c, int64_t nt) {
    // element (r, c) of a tile grid stored tile-column-major (tile (I, C) at C*nt + I)
    return ((c >> 6) * nt + (r >> 6)) * TE + (c & 63) * TS + (r & 63);
}

// One wavefront per node row: lane l takes values l, l + 64, ... of the row's
// 3x3 blocks (coarse reads), writing those whose column node lies in the same
// grain into the lower tiles of the grain's block; every element has one writer.
__global__ void __launch_bounds__(256) gather_grain_kernel(FineCsr A, GrainGather g, const double *__restrict__ b,
                                                           double *__restrict__ arena) {
    const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (v >= A.n_nodes) return;
    const int32_t m = g.node_gmat[v];
    if (m < 0) return;
    const int64_t lv = g.node_local[v];
    double *T = arena + g.mat_aoff[m];
    const int64_t p0 = A.row_ptr[v], nv = 9 * (A.row_ptr[v + 1] - p0);
    for (int64_t e = lane; e < nv; e += 64) {
        const int32_t w = A.col[p0 + e / 9];
        if (g.node_gmat[w] != m) continue;
        const int j = (int)(e % 9);
        const int64_t r = 3 * lv + j / 3, c = 3 * (int64_t)g.node_local[w] + j % 3;
        if ((r >> 6) >= (c >> 6)) T[tile_elem(r, c)] = A.val[9 * p0 + e];
    }
    const int32_t cc = g.mat_corrcol[m];
    if (cc >= 0 && b && lane < 3) {
        double *R = arena + g.mat_roff[m];
        R[rect_elem(3 * lv + lane, cc, g.mat_nt[m])] = b[3 * v + lane];
    }
}
void launch_gather_grain_blocks(const FineCsr &A, const GrainGather &g, const double *b, double *arena,
                                hipStream_t s) {
    if (A.n_nodes <= 0) return;
    hipLaunchKernelGGL(gather_grain_kernel, dim3((unsigned)((A.n_nodes + 3) / 4)), dim3(256), 0, s, A, g, b, arena);
}

template <class T>
__global__ void set_ones_kernel(const int64_t *__restrict__ off, int64_t n, T *__restrict__ arena) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) arena[off[i]] = T(1);
}
void launch_set_ones(const int64_t *off, int64_t n, double *arena, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(set_ones_kernel<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, off, n, arena);
}
// one work-group per run, 16-byte stores
__global__ void __launch_bounds__(256) zero_runs_kernel(const int64_t *__restrict__ runs, double *arena) {
    const int64_t off = runs[2 * (int64_t)blockIdx.x], len = runs[2 * (int64_t)blockIdx.x + 1];
    double2 *p = reinterpret_cast<double2 *>(arena + off);
    for (int64_t i = threadIdx.x; i < len / 2; i += 256) p[i] = double2{0.0, 0.0};
}
void launch_zero_runs(const int64_t *runs, int64_t nruns, double *arena, hipStream_t s) {
    if (nruns <= 0) return;
    hipLaunchKernelGGL(zero_runs_kernel, dim3((unsigned)nruns), dim3(256), 0, s, runs, arena);
}
template <class T>
void launch_set_ones_t(const int64_t *off, int64_t n, T *arena, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(set_ones_kernel<T>, dim3(blocks_for(n, 256)), dim3(256), 0, s, off, n, arena);
}
template void launch_set_ones_t<float>(const int64_t *, int64_t, float *, hipStream_t);
template void launch_set_ones_t<double>(const int64_t *, int64_t, double *, hipStream_t);

__global__ void gather_abar_kernel(FineCsr A, const AbarWork *__restrict__ work, int64_t nwork, CoarseMaps cm,
                                   GrainGather g, double *__restrict__ arena) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nwork) return;
    const AbarWork wk = work[i];
    const int32_t nu = cm.iface_nu[wk.c];
    const double *H = cm.H + cm.iface_hoff[wk.c];
    double *R = arena + g.mat_roff[wk.m];
    const int64_t nt = g.mat_nt[wk.m];
    const int64_t k3 = 3 * (int64_t)nu;
    for (int a = 0; a < nu; ++a) {
        double acc[9];   // acc[3 gi + di]: row gi of the node, column 3 a + di
        for (int j = 0; j < 9; ++j) acc[j] = 0.0;
        for (int64_t p = A.row_ptr[wk.v]; p < A.row_ptr[wk.v + 1]; ++p) {
            const int32_t w = A.col[p];
            if (cm.node_iface[w] != wk.c) continue;
            if (!cm.general) {
                const double h = H[(int64_t)cm.node_irow[w] * nu + a];
                for (int j = 0; j < 9; ++j) acc[j] += A.val[9 * p + j] * h;
            } else {
                const double *Mw = H + 3 * (int64_t)cm.node_irow[w] * k3 + 3 * a;   // rows 3 w + d, columns 3 a + di
                for (int gi = 0; gi < 3; ++gi)
                    for (int di = 0; di < 3; ++di) {
                        double t = 0.0;
                        for (int d = 0; d < 3; ++d) t += A.val[9 * p + 3 * gi + d] * Mw[d * k3 + di];
                        acc[3 * gi + di] += t;
                    }
            }
        }
        for (int gi = 0; gi < 3; ++gi)
            for (int di = 0; di < 3; ++di)
                R[rect_elem(3 * (int64_t)wk.lrow + gi, wk.lcol0 + 3 * a + di, nt)] = -acc[3 * gi + di];
    }
}
void launch_gather_abar(const FineCsr &A, const AbarWork *work, int64_t nwork, const CoarseMaps &cm,
                        const GrainGather &g, double *arena, hipStream_t s) {
    if (nwork <= 0) return;
    hipLaunchKernelGGL(gather_abar_kernel, dim3(blocks_for(nwork, 128)), dim3(128), 0, s, A, work, nwork, cm, g,
                       arena);
}

// One wavefront per (node, contact grid) item, lanes over the row's values as
// in the grain gather; a column node's position in the grid comes from its
// (short) list of grid memberships.
__global__ void __launch_bounds__(256) gather_contact_kernel(FineCsr A, ContactGather cg, int64_t nitems,
                                                             double *__restrict__ arena) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= nitems) return;
    const int32_t v = cg.item_node[i], m = cg.item_mat[i];
    const int64_t lv = cg.item_local[i];
    double *T = arena + cg.mat_aoff[m];
    const int64_t p0 = A.row_ptr[v], nv = 9 * (A.row_ptr[v + 1] - p0);
    for (int64_t e = lane; e < nv; e += 64) {
        const int32_t w = A.col[p0 + e / 9];
        int64_t lw = -1;
        for (int64_t q = cg.node_cptr[w]; q < cg.node_cptr[w + 1]; ++q)
            if (cg.node_cmat[q] == m) {
                lw = cg.node_cloc[q];
                break;
            }
        if (lw < 0) continue;
        const int j = (int)(e % 9);
        const int64_t r = 3 * lv + j / 3, c = 3 * lw + j % 3;
        if ((r >> 6) >= (c >> 6)) T[tile_elem(r, c)] = A.val[9 * p0 + e];
    }
}
void launch_gather_contact_blocks(const FineCsr &A, const ContactGather &c, int64_t nitems, double *arena,
                                  hipStream_t s) {
    if (nitems <= 0) return;
    hipLaunchKernelGGL(gather_contact_kernel, dim3((unsigned)((nitems + 3) / 4)), dim3(256), 0, s, A, c, nitems,
                       arena);
}

// ---- coarse Galerkin assembly ----------------------------------------------------
// element (r, c) of a symmetric front stored as packed lower tiles: the value
// goes to (max, min) by tile; inside a diagonal tile both triangles are kept
__device__ __forceinline__ void sym_put(double *F, int64_t r, int64_t c, double v, bool mirror_same_tile, bool add) {
    if ((r >> 6) < (c >> 6)) {
        const int64_t t = r;
        r = c;
        c = t;
    }
    if ((r >> 6) > (c >> 6)) {
        if (add) F[tile_elem(r, c)] += v; else F[tile_elem(r, c)] = v;
    } else {
        if (add) F[tile_elem(r, c)] += v; else F[tile_elem(r, c)] = v;
        if (mirror_same_tile && r != c) {
            if (add) F[tile_elem(c, r)] += v; else F[tile_elem(c, r)] = v;
        }
    }
}

// the staged path of the coarse assembly: up to 4 mortar nodes per interface
// (its LDS then lets 18 work-groups share a CU); more take the plain path
constexpr int CA_MAXNU = 4;
constexpr int CA_PER = ((3 * CA_MAXNU) * (3 * CA_MAXNU) + 63) / 64;   // entries per thread

__global__ void __launch_bounds__(64) coarse_assemble_kernel(const CoarsePair *__restrict__ pairs,
                                                             const CoarseEdge *__restrict__ edges,
                                                             const CoarseKRef *__restrict__ krefs, CoarseMaps cm,
                                                             const double *__restrict__ bval,
                                                             const double *__restrict__ karena,
                                                             double *__restrict__ F, double *__restrict__ vals) {
    const CoarsePair pr = pairs[blockIdx.x];
    const int32_t nu1 = cm.iface_nu[pr.c], nu2 = cm.iface_nu[pr.c2];
    const int n1 = 3 * nu1, n2 = 3 * nu2;
    const double *H1 = cm.H + cm.iface_hoff[pr.c];
    const double *H2 = cm.H + cm.iface_hoff[pr.c2];
    if (!cm.general && nu1 <= CA_MAXNU && nu2 <= CA_MAXNU) {
        // Gaussian mortars: the pair's edges pass through LDS 64 at a time
        // (their weight rows and 3x3 blocks), each thread keeping the sums of
        // its entries in registers; every sum runs over the edges in order
        __shared__ double sh1[64][CA_MAXNU], sh2[64][CA_MAXNU], sb[64][9];
        const int ne = n1 * n2;
        double acc[CA_PER];
        int ia[CA_PER], ib[CA_PER], ig[CA_PER];
#pragma unroll
        for (int u = 0; u < CA_PER; ++u) {
            const int e = threadIdx.x + 64 * u, i = e / n2, j = e - (e / n2) * n2;
            acc[u] = 0.0;
            ia[u] = i / 3;
            ib[u] = j / 3;
            ig[u] = 3 * (i % 3) + j % 3;
        }
        for (int32_t c0 = 0; c0 < pr.e_count; c0 += 64) {
            const int cnt = pr.e_count - c0 < 64 ? pr.e_count - c0 : 64;
            __syncthreads();   // the previous chunk is consumed
            if ((int)threadIdx.x < cnt) {
                const CoarseEdge ed = edges[pr.e_start + c0 + threadIdx.x];
                for (int a = 0; a < nu1; ++a) sh1[threadIdx.x][a] = H1[(int64_t)ed.rv * nu1 + a];
                for (int b2 = 0; b2 < nu2; ++b2) sh2[threadIdx.x][b2] = H2[(int64_t)ed.rw * nu2 + b2];
                for (int j = 0; j < 9; ++j) sb[threadIdx.x][j] = bval[9 * ed.blk + j];
            }
            __syncthreads();
            for (int k = 0; k < cnt; ++k)
#pragma unroll
                for (int u = 0; u < CA_PER; ++u)
                    if ((int)threadIdx.x + 64 * u < ne) acc[u] += sh1[k][ia[u]] * sh2[k][ib[u]] * sb[k][ig[u]];
        }
#pragma unroll
        for (int u = 0; u < CA_PER; ++u) {
            const int e = threadIdx.x + 64 * u;
            if (e >= ne) break;
            const int i = e / n2, j = e - (e / n2) * n2;
            double kk = 0.0;
            for (int32_t k = 0; k < pr.k_count; ++k) {
                const CoarseKRef kr = krefs[pr.k_start + k];
                int64_t R = kr.lc + i, C = kr.lc2 + j;
                if (R < C) {
                    const int64_t t = R;
                    R = C;
                    C = t;
                }
                kk += karena[kr.koff + tile_elem(R, C)];
            }
            const double val = acc[u] - kk;
            vals[pr.v_off + e] = val;
            if (pr.c != pr.c2 || i >= j) sym_put(F + pr.f_off, pr.pos1 + i, pr.pos2 + j, val, true, false);
        }
        return;
    }
    for (int e = threadIdx.x; e < n1 * n2; e += 64) {
        const int i = e / n2, j = e - (e / n2) * n2;
        const int a = i / 3, gi = i % 3, bb = j / 3, di = j % 3;
        double acc = 0.0;
        if (!cm.general) {
            for (int32_t k = 0; k < pr.e_count; ++k) {
                const CoarseEdge ed = edges[pr.e_start + k];
                acc += H1[(int64_t)ed.rv * nu1 + a] * H2[(int64_t)ed.rw * nu2 + bb] * bval[9 * ed.blk + 3 * gi + di];
            }
        } else {
            // sum over the edge's 3x3 block: M1[(rv, d1), i] A[d1][d2] M2[(rw, d2), j]
            for (int32_t k = 0; k < pr.e_count; ++k) {
                const CoarseEdge ed = edges[pr.e_start + k];
                const double *m1 = H1 + 3 * (int64_t)ed.rv * n1 + i;
                const double *m2 = H2 + 3 * (int64_t)ed.rw * n2 + j;
                const double *blk = bval + 9 * ed.blk;
                for (int d1 = 0; d1 < 3; ++d1) {
                    double t = 0.0;
                    for (int d2 = 0; d2 < 3; ++d2) t += blk[3 * d1 + d2] * m2[d2 * n2];
                    acc += m1[d1 * n1] * t;
                }
            }
        }
        double kk = 0.0;
        for (int32_t k = 0; k < pr.k_count; ++k) {
            const CoarseKRef kr = krefs[pr.k_start + k];
            int64_t R = kr.lc + i, C = kr.lc2 + j;
            if (R < C) {
                const int64_t t = R;
                R = C;
                C = t;
            }
            kk += karena[kr.koff + tile_elem(R, C)];
        }
        const double val = acc - kk;
        vals[pr.v_off + e] = val;
        // S[p][q] for p in c, q in c2; a diagonal block (c == c2) is written from
        // its lower triangle only, so both triangles hold identical values
        if (pr.c != pr.c2 || i >= j) sym_put(F + pr.f_off, pr.pos1 + i, pr.pos2 + j, val, true, false);
    }
}
void launch_coarse_assemble(const CoarsePair *pairs, int64_t npairs, const CoarseEdge *edges,
                            const CoarseKRef *krefs, const CoarseMaps &cm, const double *bsr_val,
                            const double *karena, double *farena, double *vals, hipStream_t s) {
    if (npairs <= 0) return;
    hipLaunchKernelGGL(coarse_assemble_kernel, dim3((unsigned)npairs), dim3(64), 0, s, pairs, edges, krefs, cm,
                       bsr_val, karena, farena, vals);
}

// ---- multifrontal extend-add ---------------------------------------------------------
// One work-group per parent tile, both children in one launch: each parent
// element is read and written once, and its two additions come in child
// order.  Consecutive threads take consecutive rows of a tile column (the
// stored order); their child rows are mostly consecutive too.
__global__ void __launch_bounds__(256) extend_add_kernel(const ExtendTile *__restrict__ tiles,
                                                         const int32_t *__restrict__ inv, double *arena) {
    const ExtendTile w = tiles[blockIdx.x];
    double *P = arena + w.parent_off;
#pragma unroll 4
    for (int q = 0; q < TE / 256; ++q) {
        const int e = threadIdx.x + 256 * q;
        const int64_t pr = (int64_t)w.PI * TS + (e & (TS - 1)), pc = (int64_t)w.PJ * TS + (e >> 6);
        double v = 0.0;
        bool hit = false;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (w.child_off[s] < 0) continue;
            const int32_t a = inv[w.inv_off[s] + pr], b = inv[w.inv_off[s] + pc];
            if (a < 0 || b < 0) continue;
            const int32_t hi = a > b ? a : b, lo = a > b ? b : a;
            const double c = arena[w.child_off[s] + tri_index(w.nt_d[s] + (hi >> 6), w.nt_d[s] + (lo >> 6)) * TE +
                                   (int64_t)(lo & (TS - 1)) * TS + (hi & (TS - 1))];
            if (!hit) v = P[e];
            hit = true;
            v += c;
        }
        if (hit) P[e] = v;
    }
}
void launch_extend_add(const ExtendTile *tiles, int64_t ntiles, const int32_t *inv, double *arena, hipStream_t s) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(extend_add_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, tiles, inv, arena);
}

__global__ void gather_add_kernel(const int64_t *__restrict__ dst_idx, const int64_t *__restrict__ ptr,
                                  const int64_t *__restrict__ src_idx, int64_t n, const double *src, double *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) s += src[src_idx[q]];
    dst[dst_idx[i]] += s;
}
void launch_gather_add(const int64_t *dst_idx, const int64_t *ptr, const int64_t *src_idx, int64_t n,
                       const double *src, double *dst, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(gather_add_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, dst_idx, ptr, src_idx, n, src, dst);
}

__global__ void copy_idx_kernel(const int64_t *__restrict__ dst_idx, const int64_t *__restrict__ src_idx, int64_t n,
                                const double *src, double *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[dst_idx[i]] = src[src_idx[i]];
}
void launch_copy_idx(const int64_t *dst_idx, const int64_t *src_idx, int64_t n, const double *src, double *dst,
                     hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(copy_idx_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, dst_idx, src_idx, n, src, dst);
}

__global__ void gather_scalar_kernel(const int64_t *__restrict__ off, int64_t n, const double *__restrict__ src,
                                     double *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[off[i]];
}
void launch_gather_scalar(const int64_t *off, int64_t n, const double *src, double *dst, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(gather_scalar_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, off, n, src, dst);
}

// ---- conversions ------------------------------------------------------------------
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__global__ void cvt_f64_f32_kernel(const double *__restrict__ s, float *__restrict__ d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (float)s[i];
}
__global__ void cvt_f32_bf16_kernel(const float *__restrict__ s, uint16_t *__restrict__ d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = f32_to_bf16_rne(s[i]);
}
__global__ void cvt_f64_bf16_kernel(const double *__restrict__ s, uint16_t *__restrict__ d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = f32_to_bf16_rne((float)s[i]);
}
void launch_convert_f64_f32(const double *src, float *dst, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(cvt_f64_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, dst, n);
}
void launch_convert_f32_bf16(const float *src, uint16_t *dst, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(cvt_f32_bf16_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, dst, n);
}
void launch_convert_f64_bf16(const double *src, uint16_t *dst, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(cvt_f64_bf16_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, dst, n);
}

// ---- streaming triad (bandwidth reference) -------------------------------------------
// a = b + s c over n doubles: one 16-byte load of b and of c and one 16-byte
// store per thread and as many work-groups as that takes (a grid-stride loop
// only past 2^30 work-groups).  Two reads and one write per element.  On the
// MI355X this flat form measured 6.1 TB/s with 1 GiB arrays, against
// 4.3-5.4 TB/s for grids of 1 024-32 768 work-groups looping four or one
// vectors per thread, with or without non-temporal accesses.
__global__ void __launch_bounds__(256) triad_kernel(double *__restrict__ a, const double *__restrict__ b,
                                                    const double *__restrict__ c, double sc, int64_t n) {
    const int64_t n2 = n / 2, stride = (int64_t)gridDim.x * blockDim.x;
    double2 *a2 = reinterpret_cast<double2 *>(a);
    const double2 *b2 = reinterpret_cast<const double2 *>(b), *c2 = reinterpret_cast<const double2 *>(c);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) {
        const double2 bv = b2[i], cv = c2[i];
        a2[i] = double2{bv.x + sc * cv.x, bv.y + sc * cv.y};
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) a[n - 1] = b[n - 1] + sc * c[n - 1];
}
void launch_triad(double *a, const double *b, const double *c, double sc, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>(std::max<int64_t>((n / 2 + 255) / 256, 1), (int64_t)1 << 30);
    hipLaunchKernelGGL(triad_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, b, c, sc, n);
}

// ---- Krylov --------------------------------------------------------------------------
// Every block owns KR_ROWS * 256 consecutive rows; thread t holds rows
// base + t + 256 r.  Partial sums are reduced in a fixed order (per thread,
// wave butterfly, waves 0..3, then blocks in the reduction kernel), so the
// results are bitwise reproducible.
constexpr int KR_ROWS = 2;
constexpr int KR_MAXK = 128;

int32_t multidot_blocks(int64_t n) {
    const int64_t b = (n + 256 * KR_ROWS - 1) / (256 * KR_ROWS);
    return (int32_t)(b < 1 ? 1 : b);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One pass over the block's rows of a Krylov basis:
//   x = w - sum_{j < k_sub} hsub[j] V_j      (k_sub may be 0; x written to wout if given)
//   part[b * k_dot + j] = sum_rows x . D_j   (D_j = D + j * ld_d), or x . x when D is null
// The subtraction streams four basis vectors at a time; the dot products go
// in chunks of eight vectors: every thread accumulates its rows for the
// chunk, one LDS transpose hands each vector to 32 lanes, and a 32-lane
// butterfly finishes it (one reduction per chunk instead of one per vector).
__global__ void __launch_bounds__(256) kr_pass_kernel(const double *__restrict__ V, int64_t ld, int32_t k_sub,
                                                      const double *__restrict__ hsub, const double *w,
                                                      double *wout, int64_t n, const double *__restrict__ D,
                                                      int64_t ld_d, int32_t k_dot, double *__restrict__ part) {
    __shared__ double hs[KR_MAXK];
    __shared__ double red[8][256];
    for (int j = threadIdx.x; j < k_sub; j += 256) hs[j] = hsub[j];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (256 * KR_ROWS) + threadIdx.x;
    double x[KR_ROWS];
#pragma unroll
    for (int r = 0; r < KR_ROWS; ++r) {
        const int64_t i = base + 256 * r;
        x[r] = i < n ? w[i] : 0.0;
    }
    if (k_sub > 0) {
        int32_t j = 0;
        for (; j + 4 <= k_sub; j += 4) {
#pragma unroll
            for (int r = 0; r < KR_ROWS; ++r) {
                const int64_t i = base + 256 * r;
                if (i < n) {
                    const double a0 = V[(j + 0) * ld + i], a1 = V[(j + 1) * ld + i];
                    const double a2 = V[(j + 2) * ld + i], a3 = V[(j + 3) * ld + i];
                    x[r] -= hs[j] * a0;
                    x[r] -= hs[j + 1] * a1;
                    x[r] -= hs[j + 2] * a2;
                    x[r] -= hs[j + 3] * a3;
                }
            }
        }
        for (; j < k_sub; ++j)
#pragma unroll
            for (int r = 0; r < KR_ROWS; ++r) {
                const int64_t i = base + 256 * r;
                if (i < n) x[r] -= hs[j] * V[j * ld + i];
            }
        if (wout) {
#pragma unroll
            for (int r = 0; r < KR_ROWS; ++r) {
                const int64_t i = base + 256 * r;
                if (i < n) wout[i] = x[r];
            }
        }
    }
    const int t = threadIdx.x;
    for (int32_t c = 0; c < k_dot; c += 8) {
        const int m = k_dot - c < 8 ? k_dot - c : 8;
        double acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            acc[q] = 0.0;
            if (q < m) {
                if (D) {
                    const double *d = D + (c + q) * ld_d;
#pragma unroll
                    for (int r = 0; r < KR_ROWS; ++r) {
                        const int64_t i = base + 256 * r;
                        if (i < n) acc[q] += x[r] * d[i];
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < KR_ROWS; ++r) acc[q] += x[r] * x[r];
                }
            }
        }
        __syncthreads();   // the previous chunk's reads of red are done
#pragma unroll
        for (int q = 0; q < 8; ++q) red[q][t] = acc[q];
        __syncthreads();
        const int q = t >> 5, l = t & 31;
        double sq = 0.0;
#pragma unroll
        for (int z = 0; z < 8; ++z) sq += red[q][l + 32 * z];
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
        if (l == 0 && q < m) part[(int64_t)blockIdx.x * k_dot + c + q] = sq;
    }
}
void launch_kr_pass(const double *V, int64_t ld, int32_t k_sub, const double *hsub, const double *w, double *wout,
                    int64_t n, const double *D, int64_t ld_d, int32_t k_dot, double *part, hipStream_t s) {
    hipLaunchKernelGGL(kr_pass_kernel, dim3(multidot_blocks(n)), dim3(256), 0, s, V, ld, k_sub, hsub, w, wout, n, D,
                       ld_d, k_dot, part);
}

// out[j] = sum_b part[b * k + j]; addto[j] += the same when addto is given.
__global__ void __launch_bounds__(256) kr_reduce_kernel(const double *__restrict__ part, int32_t nb, int32_t k,
                                                        double *__restrict__ out, double *__restrict__ addto) {
    __shared__ double sh[4];
    const int j = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) v += part[(int64_t)b * k + j];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = ((sh[0] + sh[1]) + sh[2]) + sh[3];
        out[j] = t;
        if (addto) addto[j] += t;
    }
}
void launch_kr_reduce(const double *part, int32_t nblocks, int32_t k, double *out, double *addto, hipStream_t s) {
    hipLaunchKernelGGL(kr_reduce_kernel, dim3(k), dim3(256), 0, s, part, nblocks, k, out, addto);
}

__global__ void add_comb_kernel(const double *__restrict__ Z, int64_t ld, int32_t k, const double *__restrict__ y,
                                double *__restrict__ x, int64_t n) {
    __shared__ double ys[128];
    for (int j = threadIdx.x; j < k; j += blockDim.x) ys[j] = y[j];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int32_t j = 0; j < k; ++j) s += Z[j * ld + i] * ys[j];
    x[i] += s;
}
void launch_add_combination(const double *Z, int64_t ld, int32_t k, const double *y, double *x, int64_t n,
                            hipStream_t s) {
    hipLaunchKernelGGL(add_comb_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, Z, ld, k, y, x, n);
}

__global__ void normalize_kernel(const double *w, const double *__restrict__ nrm2, double *v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double nr = sqrt(nrm2[0]);
    v[i] = nr > 0.0 ? w[i] / nr : 0.0;
}
void launch_normalize(const double *w, const double *nrm2, double *v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(normalize_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, w, nrm2, v, n);
}

__global__ void axpby_kernel(double a, const double *__restrict__ x, double b, const double *__restrict__ y,
                             double *__restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}
void launch_axpby(double a, const double *x, double b, const double *y, double *out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(axpby_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, a, x, b, y, out, n);
}

}  // namespace hplmm
