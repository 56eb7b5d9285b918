// Batched dense tile kernels of libhplmm (declarations shared by the host
// planner and the kernel file).
//
// Dense matrices are stored as 64x64 tiles, each tile contiguous and
// column-major (element (r, c) of a tile at c*64 + r).  Symmetric and lower
// triangular matrices keep only their lower tiles, packed: tile (I, J), I >= J,
// at index I*(I+1)/2 + J.  Every tile of every batched matrix lives in one
// "arena" buffer per element type and is addressed by an element offset.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hplmm {

constexpr int TS = 64;          // tile edge
constexpr int TE = TS * TS;     // elements per tile

__host__ __device__ inline int64_t tri_tiles(int64_t nt) { return nt * (nt + 1) / 2; }
__host__ __device__ inline int64_t tri_index(int64_t I, int64_t J) { return I * (I + 1) / 2 + J; }

enum GemmFlags : int32_t {
    GF_TRANS_A = 1,     // use op(A) = A^T
    GF_TRANS_B = 2,     // use op(B) = B^T
    GF_ACCUM = 4,       // C += alpha * sum (else C = alpha * sum)
    GF_NEGATE = 8,      // alpha = -1 (else +1)
    GF_POST = 16,       // C = alpha * P * sum, P = tile at post_off (no accumulate)
    GF_POST_RIGHT = 32, // C = ([C +] alpha * sum) * P, P = tile at post_off
};

// One output tile: C(c_off) (op)= alpha * [P *] sum_p op(A_p) op(B_p) [* P],
// and, when t_off >= 0 (tasks that do not accumulate into C), its transpose
// at t_off as well.  A long sum may be split into nchunk tasks over
// consecutive parts of its pair list (same c_off, post_off, t_off and flags,
// transposition aside): each stores its partial sum in
// part[part_off + 4096 chunk ..], and a finishing pass after the launch adds
// the partials in chunk order and applies the epilogue.
struct GemmTask {
    int64_t c_off;
    int64_t post_off;
    int32_t pair_start;
    int32_t pair_count;
    int32_t flags;
    int32_t pad;
    int64_t part_off = 0;
    int32_t pad2 = 0;
    int16_t chunk = 0;
    int16_t nchunk = 1;
    int64_t t_off = -1;
};

struct GemmPair {
    int64_t a_off;
    int64_t b_off;
};

// Diagonal-tile factorisation: A(a_off) = L L^T in place (upper part zeroed),
// W(w_off) = L^-1, Wt(wt_off) = L^-T.  `id` is reported on a bad pivot.  With
// p_off >= 0 the tile P at p_off is first subtracted as A -= P P^T (the last
// term of a left-looking diagonal update).
struct DiagTask {
    int64_t a_off;
    int64_t w_off;
    int64_t wt_off;
    int32_t id;
    int32_t pad;
    int64_t p_off = -1;
};

// Tiled matrix-vector product: y[y_off .. +64) = [base[base_off .. +64) +] sum_p T_p x[x_off_p .. +64)
// (no base term when base_off < 0).  A long row may be split into nchunk
// tasks (one work-group each) that share y_off and base_off and cover
// consecutive parts of its pair list: each writes its partial sum to
// part[part_off + 64 chunk ..], and a reduction launch after the product
// adds the partials in chunk order, then the base, and writes y.
struct GemvTask {
    int64_t y_off;
    int32_t pair_start;
    int32_t pair_count;
    int64_t base_off;
    int64_t part_off = 0;
    int16_t chunk = 0;
    int16_t nchunk = 1;
};

struct GemvPair {
    int64_t t_off;
    int64_t x_off;
};

struct CopyTask {  // dst tile = src tile^T
    int64_t src_off;
    int64_t dst_off;
};

// y = S x for a batch of symmetric matrices stored as their lower tiles, each
// tile read once.  A task (a GemvTask) is one tile row i of one matrix; its
// pairs are the tiles S_ij, j <= i.  Pair j adds S_ij x_j to y_i and, below
// the diagonal (p_off >= 0), writes the 64 values of S_ij^T x_i, the part of
// row j carried by this tile, to part[p_off ..).
struct SymPair {
    int64_t t_off;
    int64_t x_off;
    int64_t p_off;   // -1 on the diagonal
    // valid rows and columns of the tile (the last tile row and column of a
    // matrix hold fewer): the padding beyond them is never read
    int32_t rows;
    int32_t cols;
};

// Row j of the symmetric product: y[y_off + r] += sum_k part[p_off + 64 k + r]
// for k < count, in ascending k (fixed order: reproducible sums).
struct SymReduce {
    int64_t y_off;
    int64_t p_off;
    int32_t count;
    int32_t pad = 0;
};

// Launchers (stream-ordered, asynchronous).  `flag` points to a device int32
// pair {status bits, first bad id}.
// A list with split tasks (split = true) needs `part` (T); the finishing pass
// runs as a second launch on the same stream.
template <class T>
void launch_tile_gemm(T *arena, const GemmTask *tasks, const GemmPair *pairs, int64_t ntasks,
                      hipStream_t s, T *part = nullptr, bool split = false);
// The finishing pass alone (after a launch_tile_gemm of the same list with
// split = false).
template <class T>
void launch_tile_gemm_finish(T *arena, const GemmTask *tasks, const GemmPair *pairs, int64_t ntasks,
                             hipStream_t s, T *part);
// bfloat16 operands (their 16 bits) from `in`, FP32 accumulation and output
// to `out`; tasks without a second product (GF_POST / GF_POST_RIGHT ignored).
void launch_tile_gemm_bf16(const uint16_t *in, float *out, const GemmTask *tasks, const GemmPair *pairs,
                           int64_t ntasks, hipStream_t s, float *part = nullptr, bool split = false);
template <class T>
void launch_diag(T *arena_a, T *arena_w, T *arena_wt, const DiagTask *tasks, int64_t ntasks,
                 int32_t *flag, hipStream_t s);
template <class T>
void launch_tile_transpose(T *arena_src, T *arena_dst, const CopyTask *tasks, int64_t ntasks,
                           hipStream_t s);
// One work-group per task with `waves` (4 or 16) wavefronts splitting the
// pairs; base (needed only if some task has base_off >= 0) may alias y when
// every task reads its base at its own output rows.  Split rows need the
// partial buffer `part` and, after the launch and on the same stream,
// launch_gemv_split_reduce over the same tasks to finish them.
template <class T>
void launch_gemv(const T *arena, const double *x, double *y, const GemvTask *tasks,
                 const GemvPair *pairs, int64_t ntasks, hipStream_t s, const double *base = nullptr,
                 int32_t waves = 4, double *part = nullptr);
// The split rows of a launch_gemv launch over the same tasks: y = [base +]
// the sum of the row's partials in chunk order; rows not split are left alone.
void launch_gemv_split_reduce(const GemvTask *tasks, int64_t ntasks, const double *part, const double *base,
                              double *y, hipStream_t s);
// Symmetric-operator GEMV (S stored as T = double, float or bfloat16 bits;
// FP64 arithmetic): one work-group of `waves` (4 or 16) wavefronts per tile
// row; y receives the rows' own parts, part the transposed products of the
// tiles below the diagonal.  x and y must not alias.  launch_sym_reduce then
// adds the transposed products into y.
template <class T>
void launch_sym_gemv(const T *arena, const double *x, double *y, const GemvTask *tasks, const SymPair *pairs,
                     int64_t ntasks, double *part, int32_t waves, hipStream_t s);
void launch_sym_reduce(const SymReduce *tasks, int64_t ntasks, const double *part, double *y, hipStream_t s);

}  // namespace hplmm
