// Sparse, gather/scatter and Krylov kernels of libhplmm (launch wrappers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hplmm {

constexpr int SELL_C = 64;   // rows per SELL slice (one wavefront)

// Fine matrix in SELL-64 form: slice s holds rows 64s..64s+63; step k of a
// slice stores, for every lane (row), one 3x3 block as 9 arrays of 64 doubles
// (entry-major) and one column index.  Padding entries have zero values and
// the row's own column.
struct SellMatrix {
    int64_t n_rows;
    int32_t n_slices;
    const int64_t *slice_step;   // [n_slices+1] first step of each slice
    const int32_t *col;          // [steps*64]
    const double *val;           // [steps*9*64]
};

// y = A x (r == nullptr) or y = r - A x.
void launch_spmv(const SellMatrix &A, const double *x, const double *r, double *y, hipStream_t s);

// dst[i] = map[i] >= 0 ? src[map[i]] : 0, i < n
void launch_gather(const int64_t *map, const double *src, double *dst, int64_t n, hipStream_t s);

// out[d] = (base ? base[d] : 0) + (gslot[d] >= 0 ? g[gslot[d]] : 0) + sum_{q} c[cslot[q]]
// over q in [cptr[d], cptr[d+1]) (cptr may be null), d < n.
void launch_combine(int64_t n, const double *base, const int64_t *gslot, const double *g,
                    const int64_t *cptr, const int64_t *cslot, const double *c, double *out,
                    hipStream_t s);

// Coarse right-hand side (restriction P^T r).  For coarse index q:
//   f[fpos[q]] = [q < n_mortar] sum_{v in iface(q)} H[v, a(q)] r[3v + d(q)]
//                + sum_{p in [tptr[q], tptr[q+1])} t[tslot[p]]
struct CoarseMaps {
    int64_t n_ifaces;            // interfaces
    int64_t n_mortar;            // mortar dofs
    int64_t n_coarse;            // mortar dofs + corrections
    const int64_t *fpos;         // [n_coarse] position in the coarse vector arena
    const int32_t *q_iface;      // [n_mortar] interface of mortar dof q
    const int32_t *q_local;      // [n_mortar] q - moff(iface)
    const int64_t *iface_ptr;    // [n_ifaces+1]
    const int32_t *iface_nodes;  // interface node lists
    const int64_t *iface_hoff;   // [n_ifaces] offset of the interface's block in H
    const int32_t *iface_nu;     // [n_ifaces]
    const int64_t *iface_moff;   // [n_ifaces] first mortar dof
    const double *H;             // mortar blocks: general == 0: Gaussian H_c (N_c x nu_c,
                                 // Q^o block H_c (x) I_3); general == 1: the Q^o block
                                 // itself (3 N_c x 3 nu_c, rows 3 v + g, columns 3 a + g')
    int32_t general;
    const int64_t *tptr;         // [n_coarse+1]
    const int64_t *tslot;        // slots into the per-grain t arena
    const double *corr_d;        // [n_corr] coarse correction pivots b_i^T c_i
    const int32_t *node_iface;   // [n_nodes] interface of a node or -1
    const int32_t *node_irow;    // [n_nodes] row of the node inside its interface
};
void launch_coarse_rhs(const CoarseMaps &m, const double *r, const double *t, double *f, hipStream_t s);
// u[fpos[q]] = f[fpos[q]] / corr_d[q - n_mortar] for corrections
void launch_corr_solve(const CoarseMaps &m, const double *f, double *u, hipStream_t s);
// z[3v+g] = gslot[3v+g] >= 0 ? zl[gslot] : (Q^o u)[3v+g], Q^o from the interface blocks
void launch_prolong_nodes(const CoarseMaps &m, int64_t n_nodes, const int64_t *gslot, const double *zl,
                          const double *u, double *z, hipStream_t s);

// ---- set-up gathers -------------------------------------------------------
struct FineCsr {
    int64_t n_nodes;
    const int64_t *row_ptr;
    const int32_t *col;
    const double *val;
};
// Grain blocks: for every grain-interior node, scatter its row's blocks that
// couple to nodes of the same grain into the packed lower tiles of that
// grain's matrix; and b into the correction column of R.
struct GrainGather {
    const int32_t *node_gmat;    // [n_nodes] grain matrix of an interior node, -1 otherwise
    const int32_t *node_local;   // [n_nodes] local node index inside its grain / interface
    const int64_t *mat_aoff;     // [n_mats] arena offset of the packed tiles
    const int64_t *mat_roff;     // [n_mats] arena offset of R (tile grid nt x ntc, column of tiles major)
    const int32_t *mat_nt;       // [n_mats]
    const int32_t *mat_corrcol;  // [n_mats] column of b in R, or -1
};
void launch_gather_grain_blocks(const FineCsr &A, const GrainGather &g, const double *b, double *arena,
                                hipStream_t s);
// set arena[off[i]] = 1 (identity on padded diagonals)
void launch_set_ones(const int64_t *off, int64_t n, double *arena, hipStream_t s);
// arena[runs[2i] .. runs[2i] + runs[2i+1]) = 0 for i < nruns; offsets and
// lengths are multiples of 2 elements, lengths at most ZERO_RUN
constexpr int64_t ZERO_RUN = 8 * 4096;
void launch_zero_runs(const int64_t *runs, int64_t nruns, double *arena, hipStream_t s);
template <class T>
void launch_set_ones_t(const int64_t *off, int64_t n, T *arena, hipStream_t s);

// Abar gather: work item w = (node v, interface c, matrix m, local row, local
// column offset of c in m); R[3 lrow + g][lcol0 + 3a + d] = -sum_{w in c}
// A_vw[g][d] H[w, a].
struct AbarWork {
    int32_t v, c, m, lrow, lcol0, pad;
};
void launch_gather_abar(const FineCsr &A, const AbarWork *work, int64_t nwork, const CoarseMaps &cm,
                        const GrainGather &g, double *arena, hipStream_t s);

// Contact blocks: work item per (contact matrix m, local node ln).
struct ContactGather {
    const int32_t *item_node;    // [nitems] node
    const int32_t *item_mat;     // [nitems] contact matrix
    const int32_t *item_local;   // [nitems] local node index
    const int64_t *mat_aoff;     // [n_mats]
    const int64_t *node_cptr;    // [n_nodes+1] contacts containing a node (ascending)
    const int32_t *node_cmat;    // contact ids
    const int32_t *node_cloc;    // local index of the node in that contact
};
void launch_gather_contact_blocks(const FineCsr &A, const ContactGather &c, int64_t nitems, double *arena,
                                  hipStream_t s);

// Coarse Galerkin assembly: one wavefront per interface pair (c >= c').  The
// block is written into the multifrontal front that first eliminates one of
// the two interfaces (packed lower tiles at f_off, rows pos1.. for c and
// pos2.. for c2), and its values are also kept at v_off in a flat list.
struct CoarsePair {
    int32_t c, c2;
    int64_t e_start;             // edges: BSR block index, row of v in c, row of w in c2
    int32_t e_count;
    int32_t k_count;
    int64_t k_start;             // grains sharing both interfaces (K references)
    int64_t f_off;               // front tile-arena offset
    int32_t pos1, pos2;          // positions of c and c2 inside the front
    int64_t v_off;               // offset of the (3 nu_c x 3 nu_c2) block in the value list
};
struct CoarseEdge {
    int64_t blk;
    int32_t rv, rw;
};
struct CoarseKRef {
    int64_t koff;                // arena offset of packed lower K tiles of the grain
    int32_t lc, lc2;             // local column offsets of c and c2 in the grain
};
void launch_coarse_assemble(const CoarsePair *pairs, int64_t npairs, const CoarseEdge *edges,
                            const CoarseKRef *krefs, const CoarseMaps &cm, const double *bsr_val,
                            const double *karena, double *farena, double *vals, hipStream_t s);

// Multifrontal extend-add of update matrices, one work-group per 64x64 tile
// (PI, PJ), PI >= PJ, of a parent front that a child's update matrix reaches.
// Element (p, q) of the tile (both triangles of a diagonal tile) receives,
// from child 0 and then child 1, the child's boundary-block element
// (max(a, b), min(a, b)) with a = inv[p], b = inv[q], when both are >= 0.
struct ExtendTile {
    int64_t parent_off;     // the parent tile (PI, PJ)
    int64_t child_off[2];   // child fronts (packed lower tiles); -1: adds nothing to this tile
    int64_t inv_off[2];     // parent position -> child boundary row or -1: inv[inv_off + p]
    int32_t nt_d[2];        // tiles of the child's own block (its boundary block starts there)
    int32_t PI, PJ;         // tile of the parent front
    int32_t ntp, pad;       // tiles per side of the parent front
};
void launch_extend_add(const ExtendTile *tiles, int64_t ntiles, const int32_t *inv, double *arena, hipStream_t s);
// dst[dst_idx[i]] += sum_{q in [ptr[i], ptr[i+1])} src[src_idx[q]], i < n
void launch_gather_add(const int64_t *dst_idx, const int64_t *ptr, const int64_t *src_idx, int64_t n,
                       const double *src, double *dst, hipStream_t s);
// dst[dst_idx[i]] = src[src_idx[i]], i < n
void launch_copy_idx(const int64_t *dst_idx, const int64_t *src_idx, int64_t n, const double *src, double *dst,
                     hipStream_t s);
// corr_d[j] = karena[koff[j]]
void launch_gather_scalar(const int64_t *off, int64_t n, const double *src, double *dst, hipStream_t s);

// ---- conversions ----------------------------------------------------------
void launch_convert_f64_f32(const double *src, float *dst, int64_t n, hipStream_t s);
void launch_convert_f32_bf16(const float *src, uint16_t *dst, int64_t n, hipStream_t s);
void launch_convert_f64_bf16(const double *src, uint16_t *dst, int64_t n, hipStream_t s);

// ---- bandwidth reference ----------------------------------------------------
// a = b + sc c over n doubles (16-byte aligned arrays)
void launch_triad(double *a, const double *b, const double *c, double sc, int64_t n, hipStream_t s);

// ---- Krylov -----------------------------------------------------------------
// One pass over a Krylov basis, per block of rows (multidot_blocks(n) blocks):
//   x = w - sum_{j < k_sub} hsub[j] V_j  (V_j = V + j*ld; written to wout when
//   k_sub > 0 and wout is given; wout may equal w)
//   part[b*k_dot + j] = block b's share of x . D_j (D_j = D + j*ld_d), or of
//   x . x when D is null (then k_dot must be 1).  k_sub, k_dot <= 128.
void launch_kr_pass(const double *V, int64_t ld, int32_t k_sub, const double *hsub, const double *w, double *wout,
                    int64_t n, const double *D, int64_t ld_d, int32_t k_dot, double *part, hipStream_t s);
// out[j] = sum_b part[b*k + j] in a fixed order; addto[j] += the same if given
void launch_kr_reduce(const double *part, int32_t nblocks, int32_t k, double *out, double *addto, hipStream_t s);
// w = w / sqrt(*nrm2) written to v; also copies sqrt(nrm2) to *nrm_out
void launch_normalize(const double *w, const double *nrm2, double *v, int64_t n, hipStream_t s);
// x += sum_j Z_j y[j]
void launch_add_combination(const double *Z, int64_t ld, int32_t k, const double *y, double *x, int64_t n,
                            hipStream_t s);
// v = a / beta_dev (beta_dev = sqrt(nrm2))
void launch_axpby(double a, const double *x, double b, const double *y, double *out, int64_t n,
                  hipStream_t s);

int32_t multidot_blocks(int64_t n);

}  // namespace hplmm
