// Batched dense tile kernels for gfx950 (CDNA4).
//
// All batched dense linear algebra of the set-up (Cholesky, triangular
// inversion, basis products, Galerkin products) is expressed as lists of
// 64x64 tile tasks built on the host; one launch processes one list.  The
// contraction kernel stages operand tiles through LDS in 32-deep halves and
// multiplies them on the matrix cores (v_mfma_f64_16x16x4f64 /
// v_mfma_f32_16x16x4f32), four wavefronts per 64x64 output tile, each owning
// a 32x32 quadrant.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dense.h"

namespace hplmm {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
// Output layout of one 16x16 block: register r of lane l holds row row(l>>4, r),
// column l & 15.  The FP64 and FP32 instructions interleave rows differently.
template <>
struct Mfma<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lq, int r) { return lq + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lq, int r) { return 4 * lq + r; }
};

// bfloat16 operands (stored as their 16 bits) with FP32 accumulation:
// v_mfma_f32_16x16x32_bf16 takes 8 contraction indices per lane, so one
// instruction covers a whole 32-deep staged half; the output layout is that
// of the FP32 instruction.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
template <>
struct Mfma<uint16_t> {
    typedef v4f acc_t;
    static __device__ __forceinline__ int row(int lq, int r) { return 4 * lq + r; }
};

constexpr int LD = TS + 1;  // padded LDS row length (elements)
constexpr int KH = TS / 2;  // contraction depth of one staged half

// One 64x64 operand tile held across the 256 threads of a work-group, 16
// stored elements per thread, fetched so that elements 0-7 of every thread
// hold contraction indices k < 32 and elements 8-15 hold k >= 32.  The
// contraction then stages one 32-deep half at a time: 33 KB of LDS per
// work-group instead of 66 KB, so three work-groups (the register limit)
// share a CU instead of two.  With k along the stored columns (kr = false)
// element q of thread t is stored element t + 256 q; with k along the stored
// rows (kr = true) it is row (t & 31) + 32 (q >> 3), column (t >> 5) +
// 8 (q & 7).  Both orders read whole 256-byte runs.
template <class T>
struct TileRegs {
    T v[TE / 256];
};

// Where thread t's elements of one operand live: a per-thread base plus an
// offset that depends only on q and kr (uniform over the work-group), both in
// the stored tile (g) and in the LDS half (l).
struct OpMap {
    int g, l;
    bool kr;
    __device__ __forceinline__ OpMap(bool kr_, int t)
        : g(kr_ ? (t & 31) + TS * (t >> 5) : t), l(kr_ ? (t & 31) * LD + (t >> 5) : (t >> 6) * LD + (t & 63)),
          kr(kr_) {}
    __device__ __forceinline__ int goff(int q) const { return kr ? 32 * (q >> 3) + 8 * TS * (q & 7) : 256 * q; }
    // offset in half H (q in [8 H, 8 H + 8)) of the element's slot S[k - 32 H][j]
    template <int H>
    __device__ __forceinline__ int loff(int q) const { return kr ? 8 * (q & 7) : (4 * q - KH * H) * LD; }
};

template <int H, class T>
__device__ __forceinline__ void fetch_half(TileRegs<T> &r, const T *__restrict__ src, const OpMap &om) {
    const T *s = src + om.g;
#pragma unroll
    for (int q = 8 * H; q < 8 * H + 8; ++q) r.v[q] = s[om.goff(q)];
}

// Stage half H into LDS as S[k - 32 H][j], j the operand's other index (m for
// the A operand, n for B).  Operand A enters as op(A)[m][k] and B as
// op(B)[k][n], so kr is TRANS_A for A and !TRANS_B for B.  (Element q of
// thread t has k = row (t & 31) + 32 (q >> 3) and j = column (t >> 5) +
// 8 (q & 7) when kr, k = column (t >> 6) + 4 q and j = row t & 63 otherwise.)
template <int H, class T>
__device__ __forceinline__ void stage_half(T *S, const TileRegs<T> &r, const OpMap &om) {
    T *d = S + om.l;
#pragma unroll
    for (int q = 8 * H; q < 8 * H + 8; ++q) d[om.template loff<H>(q)] = r.v[q];
}

template <class T>
__device__ __forceinline__ void mfma_half(const T *As, const T *Bs, typename Mfma<T>::acc_t acc[2][2], int lane,
                                          int wm, int wn) {
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int kk = 0; kk < KH; kk += 4) {
        const int k = kk + lk;
        const T a0 = As[k * LD + wm + lr];
        const T a1 = As[k * LD + wm + 16 + lr];
        const T b0 = Bs[k * LD + wn + lr];
        const T b1 = Bs[k * LD + wn + 16 + lr];
        acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
        acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
        acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
        acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
    }
}

template <>
__device__ __forceinline__ void mfma_half<uint16_t>(const uint16_t *As, const uint16_t *Bs, v4f acc[2][2], int lane,
                                                    int wm, int wn) {
    // lane l supplies row (A) or column (B) l & 15 at contraction indices
    // 8 (l >> 4) .. 8 (l >> 4) + 7 of the half
    const int lr = lane & 15, k0 = 8 * (lane >> 4);
    v8bf a0, a1, b0, b1;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int k = (k0 + t) * LD;
        a0[t] = __builtin_bit_cast(__bf16, As[k + wm + lr]);
        a1[t] = __builtin_bit_cast(__bf16, As[k + wm + 16 + lr]);
        b0[t] = __builtin_bit_cast(__bf16, Bs[k + wn + lr]);
        b1[t] = __builtin_bit_cast(__bf16, Bs[k + wn + 16 + lr]);
    }
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
}

// Second product of a GF_POST / GF_POST_RIGHT task, half H: the accumulated
// sum leaves the registers 32 contraction indices at a time.  For C = alpha
// P S the sum is the B operand (k = its row m), held by the waves of one row
// of the 2x2 wave grid; for C = ([C +] alpha S) P the bracket is the A
// operand (k = its column n), held by the waves of one column.
template <int H, class T>
__device__ __forceinline__ void post_half(T *As, T *Bs, const T *C, const T *P, typename Mfma<T>::acc_t acc[2][2],
                                          typename Mfma<T>::acc_t res[2][2], bool left, bool acc_c, T alpha,
                                          int lane, int wm, int wn) {
    const int lr = lane & 15, lq = lane >> 4;
    const OpMap kp(!left, threadIdx.x);
    TileRegs<T> rp;
    fetch_half<H>(rp, P, kp);
    __syncthreads();
    if ((left ? wm : wn) == KH * H) {
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int r = 0; r < 4; ++r) {
                    const int m = wm + 16 * i + Mfma<T>::row(lq, r), n = wn + 16 * j + lr;
                    T v = alpha * acc[i][j][r];
                    if (left) {
                        Bs[(m - KH * H) * LD + n] = v;
                    } else {
                        if (acc_c) v += C[n * TS + m];
                        As[(n - KH * H) * LD + m] = v;
                    }
                }
    }
    stage_half<H>(left ? As : Bs, rp, kp);
    __syncthreads();
    mfma_half<T>(As, Bs, res, lane, wm, wn);
}

// The pairs of one task, accumulated into acc.  One half of each operand is
// held in registers at a time; its fetch overlaps the matrix-core work on the
// other half, already in LDS.  KA / KB: the operands' contraction index runs
// along the stored rows (compile-time, so every offset is a constant).
template <class T, bool KA, bool KB>
__device__ __forceinline__ void gemm_pairs(const T *__restrict__ arena, const GemmPair *__restrict__ pairs,
                                           const GemmTask &tk, T *As, T *Bs, typename Mfma<T>::acc_t acc[2][2],
                                           int lane, int wm, int wn) {
    const OpMap ka(KA, threadIdx.x), kb(KB, threadIdx.x);
    TileRegs<T> ra, rb;
    if (tk.pair_count > 0) {
        const GemmPair pr = pairs[tk.pair_start];
        fetch_half<0>(ra, arena + pr.a_off, ka);
        fetch_half<0>(rb, arena + pr.b_off, kb);
    }
    for (int p = 0; p < tk.pair_count; ++p) {
        const GemmPair cur = pairs[tk.pair_start + p];
        const bool more = p + 1 < tk.pair_count;
        const GemmPair nx = pairs[tk.pair_start + (more ? p + 1 : p)];
        __syncthreads();
        stage_half<0>(As, ra, ka);
        stage_half<0>(Bs, rb, kb);
        __syncthreads();
        fetch_half<1>(ra, arena + cur.a_off, ka);
        fetch_half<1>(rb, arena + cur.b_off, kb);
        mfma_half<T>(As, Bs, acc, lane, wm, wn);
        __syncthreads();
        stage_half<1>(As, ra, ka);
        stage_half<1>(Bs, rb, kb);
        __syncthreads();
        if (more) {
            fetch_half<0>(ra, arena + nx.a_off, ka);
            fetch_half<0>(rb, arena + nx.b_off, kb);
        }
        mfma_half<T>(As, Bs, acc, lane, wm, wn);
    }
}

// Tile contraction task: the pairs in 32-deep halves, then the optional
// second product and the output.  Operands are read from `in` (element type
// Ti) and the output tile is written to `out` (type T, the accumulation type):
// Ti = T for FP64 and FP32 work on one arena; Ti = bfloat16 with T = FP32
// reads bfloat16 operands and writes FP32 results (no second product).
template <class Ti, class T>
__global__ void __launch_bounds__(256) tile_gemm_kernel(const Ti *__restrict__ in, T *__restrict__ out,
                                                        const GemmTask *__restrict__ tasks,
                                                        const GemmPair *__restrict__ pairs, T *part,
                                                        int finish) {
    // the two operand halves; together they hold one padded 64x64 tile for
    // the output staging
    __shared__ T S[2 * KH * LD];
    Ti *As = reinterpret_cast<Ti *>(S), *Bs = As + KH * LD;
    // work-groups are dealt to the 8 XCDs in turn; give each XCD a contiguous
    // slice of the list, so neighbouring tasks (which share operand tiles)
    // meet in the same L2
    const uint32_t nb = gridDim.x, b = blockIdx.x, xcd = b & 7, q = nb >> 3, r = nb & 7;
    const GemmTask tk = tasks[xcd * q + (xcd < r ? xcd : r) + (b >> 3)];
    // the finishing pass: chunk 0 of each split task sums and finishes it
    if (finish && (tk.nchunk <= 1 || tk.chunk != 0)) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    typename Mfma<Ti>::acc_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = typename Mfma<Ti>::acc_t{0, 0, 0, 0};
    // the contraction loop specialised on the fetch orders (uniform branch)
    const bool ta = tk.flags & GF_TRANS_A, tb = tk.flags & GF_TRANS_B;
    if (finish) {
    } else if (ta) {
        if (tb)
            gemm_pairs<Ti, true, false>(in, pairs, tk, As, Bs, acc, lane, wm, wn);
        else
            gemm_pairs<Ti, true, true>(in, pairs, tk, As, Bs, acc, lane, wm, wn);
    } else {
        if (tb)
            gemm_pairs<Ti, false, false>(in, pairs, tk, As, Bs, acc, lane, wm, wn);
        else
            gemm_pairs<Ti, false, true>(in, pairs, tk, As, Bs, acc, lane, wm, wn);
    }
    if (tk.nchunk > 1) {
        // partial sums in accumulator order, added by the finishing pass
        if (!finish) {
            T *pp = part + tk.part_off + (int64_t)tk.chunk * TE;
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    for (int r = 0; r < 4; ++r) pp[((i * 2 + j) * 4 + r) * 256 + threadIdx.x] = acc[i][j][r];
            return;
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = typename Mfma<T>::acc_t{0, 0, 0, 0};
        for (int c = 0; c < tk.nchunk; ++c) {
            const T *pc = part + tk.part_off + (int64_t)c * TE;
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    for (int r = 0; r < 4; ++r) acc[i][j][r] += pc[((i * 2 + j) * 4 + r) * 256 + threadIdx.x];
        }
    }
    const int lr = lane & 15, lq = lane >> 4;
    const T alpha = (tk.flags & GF_NEGATE) ? T(-1) : T(1);
    T *C = out + tk.c_off;
    bool post = false;
    if constexpr (std::is_same<Ti, T>::value) post = tk.flags & (GF_POST | GF_POST_RIGHT);
    if constexpr (std::is_same<Ti, T>::value) if (post) {
        // GF_POST: C = alpha P S, P the A operand (k along its columns);
        // GF_POST_RIGHT: C = ([C +] alpha S) P, P the B operand (k along its rows)
        const bool left = tk.flags & GF_POST;
        const bool acc_c = !left && (tk.flags & GF_ACCUM);
        typename Mfma<T>::acc_t res[2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) res[i][j] = typename Mfma<T>::acc_t{0, 0, 0, 0};
        post_half<0, T>(As, Bs, C, in + tk.post_off, acc, res, left, acc_c, alpha, lane, wm, wn);
        post_half<1, T>(As, Bs, C, in + tk.post_off, acc, res, left, acc_c, alpha, lane, wm, wn);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = res[i][j];
    }
    // stage the result column-major in LDS (both halves), then store coalesced
    __syncthreads();
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int m = wm + 16 * i + Mfma<Ti>::row(lq, r), n = wn + 16 * j + lr;
                S[n * LD + m] = acc[i][j][r];
            }
    __syncthreads();
    const T a2 = post ? T(1) : alpha;
    const bool accum = (tk.flags & GF_ACCUM) && !post;
    const int t = threadIdx.x;
#pragma unroll 4
    for (int q = 0; q < TE / 256; ++q) {
        const int e = t + 256 * q;
        const int m = e & (TS - 1), n = e >> 6;
        const T v = a2 * S[n * LD + m];
        C[e] = accum ? C[e] + v : v;
    }
    if (tk.t_off >= 0) {
        // the transposed copy, coalesced in its own order (tasks that
        // accumulate into C never ask for one)
        T *Ct = out + tk.t_off;
#pragma unroll 4
        for (int q = 0; q < TE / 256; ++q) {
            const int e = t + 256 * q;
            const int m = e & (TS - 1), n = e >> 6;   // Ct(m, n) = C(n, m)
            Ct[e] = a2 * S[m * LD + n];
        }
    }
}

// 1/d for a positive normal d.  FP64: the hardware reciprocal refined by
// two Newton-Raphson steps x <- x + x (1 - d x), within an ulp or so of the
// rounded quotient and a third of the latency of an IEEE division, which
// sits on the diagonal factorisation's serial path once per column.
template <class T>
__device__ __forceinline__ T pivot_recip(T d) {
    return T(1) / d;
}
template <>
__device__ __forceinline__ double pivot_recip<double>(double d) {
    double x = __builtin_amdgcn_rcp(d);
    double e = fma(-d, x, 1.0);
    x = fma(x, e, x);
    e = fma(-d, x, 1.0);
    return fma(x, e, x);
}

// Cholesky factor L and inverse W = L^-1 of one 64x64 tile, held in
// registers: lane r of wave q keeps row r of L and row r of V = W^T at the
// columns c = q + 4k (k < 16).  Step j uses the unscaled pivot d_j = L_jj:
// the owners of column j publish it (L and V) through LDS, then every thread
// subtracts L_rj L_cj / d_j from its entries of L and V_rj L_cj / d_j from V
// (forward elimination on the identity) for c > j.  Later steps read only
// later columns, so the scaling of column j by 1/sqrt(d_j) waits until all
// 64 steps are done (d_j is kept in LDS) and leaves the serial path.
// Entries above the diagonal of L are never read for the lower part and are
// masked on store.  One barrier per step (double-buffered columns); the
// published column is stored permuted (slot (c & 3) * 16 + c / 4) so a
// thread's 16 values are contiguous.  The 64 steps are unrolled at compile
// time so every register index is static.
template <class T, int J>
struct DiagStep {
    static __device__ __forceinline__ void run(T (&Lr)[16], T (&Vr)[16], T *colL, T *colV, T *piv, int r, int q,
                                               bool &bad) {
        constexpr int kj = J >> 2, qj = J & 3;
        T *cl = colL + (J & 1) * TS;
        T *cv = colV + (J & 1) * TS;
        const int pr = (r & 3) * 16 + (r >> 2);
        if (q == qj) {
            cl[pr] = Lr[kj];
            cv[pr] = Vr[kj];
        }
        __syncthreads();
        T d = cl[qj * 16 + kj];
        if (!(d > T(0)) || !(d < T(INFINITY))) {
            bad = true;
            d = T(1);
        }
        if (threadIdx.x == 0) piv[J] = d;
        const T inv_d = pivot_recip<T>(d);
        const T lrj = cl[pr] * inv_d;
        const T vrj = cv[pr] * inv_d;
        const T *cq = cl + q * 16;
#pragma unroll
        for (int k = kj; k < 16; ++k) {
            const T lcj = cq[k];
            if (k > kj || q > qj) {
                Lr[k] -= lrj * lcj;
                Vr[k] -= vrj * lcj;
            }
        }
        DiagStep<T, J + 1>::run(Lr, Vr, colL, colV, piv, r, q, bad);
    }
};
template <class T>
struct DiagStep<T, TS> {
    static __device__ __forceinline__ void run(T (&)[16], T (&)[16], T *, T *, T *, int, int, bool &) {}
};

template <class T>
__global__ void __launch_bounds__(256) diag_kernel(T *__restrict__ A, T *__restrict__ Wa,
                                                   T *__restrict__ Wta,
                                                   const DiagTask *__restrict__ tasks,
                                                   int32_t *__restrict__ flag) {
    __shared__ T colL[2 * TS];
    __shared__ T colV[2 * TS];
    __shared__ T piv[TS];
    __shared__ T S[TS * LD];
    const DiagTask tk = tasks[blockIdx.x];
    const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
    T *a = A + tk.a_off;
    T Lr[16], Vr[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int c = q + 4 * k;
        Lr[k] = r >= c ? a[c * TS + r] : T(0);
        Vr[k] = r == c ? T(1) : T(0);
    }
    if (tk.p_off >= 0) {
        // A -= P P^T on the matrix cores: P staged in LDS as S[k][m] = P(m, k)
        // (both operands read from it); the waves of the three lower 32x32
        // quadrants accumulate theirs over k = 0..63, the upper one idles
        // every load issued before the first store, so that they overlap
        const T *pp = A + tk.p_off;
        T pv[TE / 256];
#pragma unroll
        for (int u = 0; u < TE / 256; ++u) pv[u] = pp[threadIdx.x + 256 * u];
#pragma unroll
        for (int u = 0; u < TE / 256; ++u) {
            const int e = threadIdx.x + 256 * u;
            S[(e >> 6) * LD + (e & (TS - 1))] = pv[u];
        }
        __syncthreads();
        const int lr = r & 15, lq = r >> 4;
        const int wm = (q >> 1) * 32, wn = (q & 1) * 32;
        typename Mfma<T>::acc_t acc[2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = typename Mfma<T>::acc_t{0, 0, 0, 0};
        if (wm >= wn) {
#pragma unroll
            for (int kk = 0; kk < TS; kk += 4) {
                const int k = kk + lq;
                const T a0 = S[k * LD + wm + lr], a1 = S[k * LD + wm + 16 + lr];
                const T b0 = S[k * LD + wn + lr], b1 = S[k * LD + wn + 16 + lr];
                acc[0][0] = Mfma<T>::mac(a0, b0, acc[0][0]);
                acc[0][1] = Mfma<T>::mac(a0, b1, acc[0][1]);
                acc[1][0] = Mfma<T>::mac(a1, b0, acc[1][0]);
                acc[1][1] = Mfma<T>::mac(a1, b1, acc[1][1]);
            }
        }
        __syncthreads();   // every wave has read P
        if (wm >= wn)
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    for (int rr = 0; rr < 4; ++rr)
                        S[(wn + 16 * j + lr) * LD + wm + 16 * i + Mfma<T>::row(lq, rr)] = acc[i][j][rr];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int c = q + 4 * k;
            if (r >= c) Lr[k] -= S[c * LD + r];
        }
    }
    bool bad = false;
    DiagStep<T, 0>::run(Lr, Vr, colL, colV, piv, r, q, bad);
    // the deferred column scaling: column c of L and of V by 1/sqrt(d_c)
    __syncthreads();
    if (threadIdx.x < TS) colL[threadIdx.x] = T(1) / sqrt(piv[threadIdx.x]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const T sc = colL[q + 4 * k];
        Lr[k] *= sc;
        Vr[k] *= sc;
    }
    // L and W^T = V are stored with coalesced writes; W goes through LDS
    T *w = Wa + tk.w_off;
    T *wt = Wta + tk.wt_off;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int c = q + 4 * k;
        a[c * TS + r] = r >= c ? Lr[k] : T(0);
        wt[c * TS + r] = Vr[k];
        S[r * LD + c] = Vr[k];   // S(r, c) = W(c, r)
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TE; e += 256) {
        const int row = e & (TS - 1), col = e >> 6;
        w[e] = S[col * LD + row];
    }
    if (bad && threadIdx.x == 0) {
        atomicOr(&flag[0], 1);
        atomicMin(&flag[1], tk.id);
    }
}

template <class T>
__global__ void __launch_bounds__(256) tile_transpose_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                             const CopyTask *__restrict__ tasks) {
    __shared__ T S[TS * LD];
    const CopyTask tk = tasks[blockIdx.x];
    const int t = threadIdx.x;
    const T *s = src + tk.src_off;
    // every load issued before the first store, so that they overlap
    T v[TE / 256];
#pragma unroll
    for (int u = 0; u < TE / 256; ++u) v[u] = s[t + 256 * u];
#pragma unroll
    for (int u = 0; u < TE / 256; ++u) {
        const int e = t + 256 * u, r = e & (TS - 1), c = e >> 6;
        S[r * LD + c] = v[u];
    }
    __syncthreads();
    T *d = dst + tk.dst_off;
#pragma unroll
    for (int u = 0; u < TE / 256; ++u) {
        const int e = t + 256 * u, r = e & (TS - 1), c = e >> 6;   // dst(r, c) = src(c, r)
        d[e] = S[c * LD + r];
    }
}

// ---- tiled GEMV --------------------------------------------------------
template <class T>
struct Vec16;  // 16-byte load of consecutive tile elements, widened to double
template <>
struct Vec16<double> {
    static constexpr int R = 2;
    typedef double2 raw_t;
    static __device__ __forceinline__ raw_t load_raw(const double *p) { return *reinterpret_cast<const double2 *>(p); }
    static __device__ __forceinline__ void widen(const raw_t &v, double *o) {
        o[0] = v.x;
        o[1] = v.y;
    }
    static __device__ __forceinline__ void load(const double *p, double *o) { widen(load_raw(p), o); }
};
template <>
struct Vec16<float> {
    static constexpr int R = 4;
    typedef float4 raw_t;
    static __device__ __forceinline__ raw_t load_raw(const float *p) { return *reinterpret_cast<const float4 *>(p); }
    static __device__ __forceinline__ void widen(const raw_t &v, double *o) {
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
    static __device__ __forceinline__ void load(const float *p, double *o) { widen(load_raw(p), o); }
};
template <>
struct Vec16<uint16_t> {   // bfloat16 storage
    static constexpr int R = 8;
    typedef uint4 raw_t;
    static __device__ __forceinline__ raw_t load_raw(const uint16_t *p) { return *reinterpret_cast<const uint4 *>(p); }
    static __device__ __forceinline__ void widen(const raw_t &v, double *o) {
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = (double)__uint_as_float(w[i] << 16);
            o[2 * i + 1] = (double)__uint_as_float(w[i] & 0xffff0000u);
        }
    }
    static __device__ __forceinline__ void load(const uint16_t *p, double *o) { widen(load_raw(p), o); }
};

template <class T, int NW>
__global__ void __launch_bounds__(64 * NW) gemv_kernel(const T *__restrict__ arena, const double *__restrict__ x,
                                                       double *y, const GemvTask *__restrict__ tasks,
                                                       const GemvPair *__restrict__ pairs, const double *base,
                                                       double *part) {
    constexpr int R = Vec16<T>::R;          // rows per lane
    constexpr int LPC = TS / R;             // lanes per column
    __shared__ double red[NW * R * TS];
    const GemvTask tk = tasks[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int phase = lane / LPC, row0 = (lane % LPC) * R;
    double acc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] = 0.0;
    for (int p = wave; p < tk.pair_count; p += NW) {
        const GemvPair pr = pairs[tk.pair_start + p];
        const T *tile = arena + pr.t_off;
        const double *xs = x + pr.x_off;
#pragma unroll 8
        for (int c = phase; c < TS; c += R) {
            double v[R];
            Vec16<T>::load(tile + c * TS + row0, v);
            const double xc = xs[c];
#pragma unroll
            for (int i = 0; i < R; ++i) acc[i] += v[i] * xc;
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) red[(wave * R + phase) * TS + row0 + i] = acc[i];
    __syncthreads();
    if (threadIdx.x >= TS) return;   // wave 0 finishes the task
    const int t = threadIdx.x;
    double s = 0.0;
    for (int q = 0; q < NW * R; ++q) s += red[q * TS + t];
    if (tk.nchunk > 1) {
        // a chunk of a split row: its partial sum, added up by the reduction
        // launch that follows (a kernel boundary instead of agent-scope fences,
        // whose L2 write-back and invalidation cost more than the launch)
        part[tk.part_off + (int64_t)tk.chunk * TS + t] = s;
        return;
    }
    if (tk.base_off >= 0) s += base[tk.base_off + t];
    y[tk.y_off + t] = s;
}

// ---- symmetric-operator GEMV ----------------------------------------------
// Storage T (double, float or bfloat16); products and sums in FP64.  Lane l
// of a wave reads R = 16 / sizeof(T) consecutive rows of a tile column with
// one 16-byte load: the LPC = 64 / R lanes l % LPC cover the column, and the
// R groups l / LPC take R neighbouring columns, so each load instruction
// covers R whole columns.  The row part S_ij x_j accumulates in R registers
// over all tiles of the task.  The transposed part needs, per column, the sum
// over the LPC lanes of a group; it is formed per chunk of 8 columns per
// lane: a reduce-scatter over the top three bits of l % LPC (8 -> 4 -> 2 -> 1
// values per lane) and a butterfly over the remaining low bits leave lane l
// with column u = 4 b2 + 2 b1 + b0 of the chunk (b2 b1 b0 those three bits),
// replicated over those low bits.  The chunk count equals the number of such
// replicas, so the lane whose low bits equal the chunk keeps its value, and
// one store per tile with every lane active writes the tile's 64 slot values.
// The last tile row and column of a matrix extend past its end: their padded
// rows and columns (zero, or the identity on the diagonal, times a zero x)
// are masked off instead of read.  Of the diagonal tile S_II only the lower
// triangle is read: its rows r >= c give the row part, rows r > c the
// transposed part, reduce-scattered like the others into LDS and added to
// this row's result (the diagonal tile is the last pair of every row task).
// Tiles are read with buffer loads, whose out-of-range lanes return zeros
// without a memory access: the masks cost no branch.  Against plain loads
// with the masks as branches this measured 33.4 against 34.4 ms per step
// (FP64 S, 64^3 GRF) and 18.9 against 28.0 ms (FP32 S, where the branches
// kept each masked load's widening inside them and serialised the loads).

typedef unsigned int v4u __attribute__((ext_vector_type(4)));
constexpr int BUF_WORD3 = 0x00020000;   // buffer resource word 3 for CDNA (32-bit data format, raw access)
constexpr int BUF_OOB = 0x7ffffff0;     // a byte offset past any tile: the load returns zeros

// One tile of a row task: the row part into acc, the lane's share of the
// transposed part returned (the slot value of the chunk its low bits name).
template <class T>
__device__ __forceinline__ double sym_tile(const T *__restrict__ tile, const double *__restrict__ xs,
                                           const double (&xi)[Vec16<T>::R], double (&acc)[Vec16<T>::R], int phase,
                                           int lc, int row0, bool b2, bool b1, bool b0, int rows, int cols,
                                           bool diag) {
    constexpr int R = Vec16<T>::R, LPC = TS / R, NCH = TS / (8 * R);
    constexpr int H2 = LPC / 2, H1 = LPC / 4, H0 = LPC / 8;
    const bool rok = row0 < rows;
    // the tile as a buffer resource (byte range TE elements; raw addressing)
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(tile), 0, TE * (int)sizeof(T), BUF_WORD3);
    double mine = 0.0;
#pragma unroll 1
    for (int ch = 0; ch < NCH; ++ch) {
        double cs[8];
        // four buffer loads at a time issue first, then their x values: lanes
        // outside the valid part get an offset past the tile's end and read
        // zeros without touching memory, so no branch holds a load back
#pragma unroll
        for (int hh = 0; hh < 8; hh += 4) {
            v4u bits[4];
            double xc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = R * (8 * ch + hh + u) + phase;
                const bool ok = rok && c < cols && (!diag || row0 + R > c);
                bits[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, ok ? (c * TS + row0) * (int)sizeof(T) : BUF_OOB,
                                                                0, 0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) xc[u] = xs[R * (8 * ch + hh + u) + phase];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = R * (8 * ch + hh + u) + phase;
                double v[R];
                Vec16<T>::widen(__builtin_bit_cast(typename Vec16<T>::raw_t, bits[u]), v);
                double t = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // diagonal tile: row part from rows r >= c, transposed
                    // part from rows r > c (the upper triangle mirrors them)
                    const double vr = diag && row0 + r < c ? 0.0 : v[r];
                    acc[r] += vr * xc[u];
                    t += diag && row0 + r == c ? 0.0 : vr * xi[r];
                }
                cs[hh + u] = t;
            }
        }
        double t4[4], t3[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) t4[k] = (b2 ? cs[k + 4] : cs[k]) + __shfl_xor(b2 ? cs[k] : cs[k + 4], H2);
#pragma unroll
        for (int k = 0; k < 2; ++k) t3[k] = (b1 ? t4[k + 2] : t4[k]) + __shfl_xor(b1 ? t4[k] : t4[k + 2], H1);
        double t = (b0 ? t3[1] : t3[0]) + __shfl_xor(b0 ? t3[0] : t3[1], H0);
#pragma unroll
        for (int m = H0 / 2; m >= 1; m /= 2) t += __shfl_xor(t, m);
        if ((lc & (H0 - 1)) == ch) mine = t;
    }
    return mine;
}

template <class T, int NW>
__global__ void __launch_bounds__(64 * NW) sym_gemv_kernel(const T *__restrict__ arena,
                                                           const double *__restrict__ x, double *__restrict__ y,
                                                           const GemvTask *__restrict__ tasks,
                                                           const SymPair *__restrict__ pairs,
                                                           double *__restrict__ part) {
    constexpr int R = Vec16<T>::R;                      // rows per lane: 2, 4, 8
    constexpr int LPC = TS / R;                         // lanes per column: 32, 16, 8
    constexpr int H2 = LPC / 2, H1 = LPC / 4, H0 = LPC / 8;   // the reduce-scatter's lane bits
    __shared__ double red[NW * R * TS];
    __shared__ double dgs[TS];   // the diagonal tile's transposed part, added to this row
    const GemvTask tk = tasks[blockIdx.x];
    // the wave index is uniform: its tile pointers (and buffer resources) live in scalar registers
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int phase = lane / LPC, lc = lane % LPC, row0 = lc * R;
    const bool b2 = lc & H2, b1 = lc & H1, b0 = lc & H0;
    const int uq = 4 * (int)b2 + 2 * (int)b1 + (int)b0;
    double xi[R], acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        xi[r] = x[tk.y_off + row0 + r];
        acc[r] = 0.0;
    }
    for (int p = wave; p < tk.pair_count; p += NW) {
        const SymPair pr = pairs[tk.pair_start + p];
        const T *tile = arena + pr.t_off;
        const double *xs = x + pr.x_off;
        const bool below = pr.p_off >= 0;
        const double mine = sym_tile<T>(tile, xs, xi, acc, phase, lc, row0, b2, b1, b0, pr.rows, pr.cols, !below);
        // one store per tile with every lane active: a slot of row J, or for
        // the diagonal tile this row's own part
        const int col = R * (8 * (lc & (H0 - 1)) + uq) + phase;
        if (below)
            part[pr.p_off + col] = mine;
        else
            dgs[col] = mine;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) red[(wave * R + phase) * TS + row0 + r] = acc[r];
    __syncthreads();
    if (threadIdx.x >= TS) return;   // wave 0 finishes the row
    const int t = threadIdx.x;
    double s = 0.0;
    for (int q = 0; q < NW * R; ++q) s += red[q * TS + t];
    y[tk.y_off + t] = s + dgs[t];
}

// The split rows of a GEMV launch: one wavefront per task of the launch; the
// first chunk's wavefront adds the row's partial sums in chunk order, then the
// base, and stores the row.
__global__ void __launch_bounds__(256) gemv_split_reduce_kernel(const GemvTask *__restrict__ tasks, int64_t ntasks,
                                                                const double *__restrict__ part,
                                                                const double *base, double *y) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= ntasks) return;
    const GemvTask tk = tasks[i];
    if (tk.nchunk <= 1 || tk.chunk != 0) return;
    const int t = threadIdx.x & 63;
    double s = 0.0;
    for (int c = 0; c < tk.nchunk; ++c) s += part[tk.part_off + (int64_t)c * TS + t];
    if (tk.base_off >= 0) s += base[tk.base_off + t];
    y[tk.y_off + t] = s;
}

// One wavefront per row: lane r adds the row's transposed products in order.
__global__ void __launch_bounds__(256) sym_reduce_kernel(const SymReduce *__restrict__ tasks, int64_t ntasks,
                                                         const double *__restrict__ part, double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= ntasks) return;
    const SymReduce tk = tasks[i];
    const int r = threadIdx.x & 63;
    double s = y[tk.y_off + r];
    const double *pp = part + tk.p_off + r;
    // eight loads in flight, added in ascending k
    int32_t k = 0;
    for (; k + 8 <= tk.count; k += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = pp[(int64_t)(k + u) * TS];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; k < tk.count; ++k) s += pp[(int64_t)k * TS];
    y[tk.y_off + r] = s;
}

// ---- launchers -----------------------------------------------------------
static inline unsigned grid_of(int64_t n) { return (unsigned)n; }

template <class T>
void launch_tile_gemm(T *arena, const GemmTask *tasks, const GemmPair *pairs, int64_t ntasks, hipStream_t s,
                      T *part, bool split) {
    if (ntasks <= 0) return;
    for (int finish = 0; finish <= (split ? 1 : 0); ++finish)
        hipLaunchKernelGGL((tile_gemm_kernel<T, T>), dim3(grid_of(ntasks)), dim3(256), 0, s, arena, arena, tasks,
                           pairs, part, finish);
}
template <class T>
void launch_tile_gemm_finish(T *arena, const GemmTask *tasks, const GemmPair *pairs, int64_t ntasks, hipStream_t s,
                             T *part) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL((tile_gemm_kernel<T, T>), dim3(grid_of(ntasks)), dim3(256), 0, s, arena, arena, tasks, pairs,
                       part, 1);
}
void launch_tile_gemm_bf16(const uint16_t *in, float *out, const GemmTask *tasks, const GemmPair *pairs,
                           int64_t ntasks, hipStream_t s, float *part, bool split) {
    if (ntasks <= 0) return;
    for (int finish = 0; finish <= (split ? 1 : 0); ++finish)
        hipLaunchKernelGGL((tile_gemm_kernel<uint16_t, float>), dim3(grid_of(ntasks)), dim3(256), 0, s, in, out,
                           tasks, pairs, part, finish);
}
template <class T>
void launch_diag(T *a, T *w, T *wt, const DiagTask *tasks, int64_t ntasks, int32_t *flag, hipStream_t s) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(diag_kernel<T>, dim3(grid_of(ntasks)), dim3(256), 0, s, a, w, wt, tasks, flag);
}
template <class T>
void launch_tile_transpose(T *src, T *dst, const CopyTask *tasks, int64_t ntasks, hipStream_t s) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(tile_transpose_kernel<T>, dim3(grid_of(ntasks)), dim3(256), 0, s, src, dst, tasks);
}
template <class T>
void launch_gemv(const T *arena, const double *x, double *y, const GemvTask *tasks, const GemvPair *pairs,
                 int64_t ntasks, hipStream_t s, const double *base, int32_t waves, double *part) {
    if (ntasks <= 0) return;
    if (waves == 16)
        hipLaunchKernelGGL((gemv_kernel<T, 16>), dim3(grid_of(ntasks)), dim3(1024), 0, s, arena, x, y, tasks, pairs,
                           base, part);
    else
        hipLaunchKernelGGL((gemv_kernel<T, 4>), dim3(grid_of(ntasks)), dim3(256), 0, s, arena, x, y, tasks, pairs,
                           base, part);
}
void launch_gemv_split_reduce(const GemvTask *tasks, int64_t ntasks, const double *part, const double *base,
                              double *y, hipStream_t s) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(gemv_split_reduce_kernel, dim3((unsigned)((ntasks + 3) / 4)), dim3(256), 0, s, tasks, ntasks,
                       part, base, y);
}

template <class T>
void launch_sym_gemv(const T *arena, const double *x, double *y, const GemvTask *tasks, const SymPair *pairs,
                     int64_t ntasks, double *part, int32_t waves, hipStream_t s) {
    if (ntasks <= 0) return;
    // narrow storage needs more registers per lane than 16 waves leave: 4 waves
    if constexpr (sizeof(T) == 8) {
        if (waves == 16) {
            hipLaunchKernelGGL((sym_gemv_kernel<T, 16>), dim3(grid_of(ntasks)), dim3(1024), 0, s, arena, x, y,
                               tasks, pairs, part);
            return;
        }
    }
    hipLaunchKernelGGL((sym_gemv_kernel<T, 4>), dim3(grid_of(ntasks)), dim3(256), 0, s, arena, x, y, tasks, pairs,
                       part);
}
template void launch_sym_gemv<double>(const double *, const double *, double *, const GemvTask *, const SymPair *,
                                      int64_t, double *, int32_t, hipStream_t);
template void launch_sym_gemv<float>(const float *, const double *, double *, const GemvTask *, const SymPair *,
                                     int64_t, double *, int32_t, hipStream_t);
void launch_sym_reduce(const SymReduce *tasks, int64_t ntasks, const double *part, double *y, hipStream_t s) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(sym_reduce_kernel, dim3((unsigned)((ntasks + 3) / 4)), dim3(256), 0, s, tasks, ntasks, part,
                       y);
}

template void launch_tile_gemm<double>(double *, const GemmTask *, const GemmPair *, int64_t, hipStream_t, double *,
                                       bool);
template void launch_tile_gemm<float>(float *, const GemmTask *, const GemmPair *, int64_t, hipStream_t, float *,
                                      bool);
template void launch_tile_gemm_finish<double>(double *, const GemmTask *, const GemmPair *, int64_t, hipStream_t,
                                              double *);
template void launch_tile_gemm_finish<float>(float *, const GemmTask *, const GemmPair *, int64_t, hipStream_t,
                                             float *);
template void launch_diag<double>(double *, double *, double *, const DiagTask *, int64_t, int32_t *, hipStream_t);
template void launch_diag<float>(float *, float *, float *, const DiagTask *, int64_t, int32_t *, hipStream_t);
template void launch_tile_transpose<double>(double *, double *, const CopyTask *, int64_t, hipStream_t);
template void launch_tile_transpose<float>(float *, float *, const CopyTask *, int64_t, hipStream_t);
template void launch_gemv<double>(const double *, const double *, double *, const GemvTask *, const GemvPair *,
                                  int64_t, hipStream_t, const double *, int32_t, double *);
template void launch_gemv<float>(const float *, const double *, double *, const GemvTask *, const GemvPair *,
                                 int64_t, hipStream_t, const double *, int32_t, double *);
template void launch_gemv<uint16_t>(const uint16_t *, const double *, double *, const GemvTask *,
                                    const GemvPair *, int64_t, hipStream_t, const double *, int32_t, double *);

}  // namespace hplmm
