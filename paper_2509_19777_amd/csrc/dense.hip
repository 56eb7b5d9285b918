// Batched dense tile kernels for gfx950 (CDNA4).
//
// All batched dense linear algebra of the set-up (Cholesky, triangular
// inversion, basis products, Galerkin products) is expressed as lists of
// 64x64 tile tasks built on the host; one launch processes one list.  The
// contraction kernel stages operand tiles through LDS and multiplies them on
// the matrix cores (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32), four
// wavefronts per 64x64 output tile, each owning a 32x32 quadrant.
#include <hip/hip_runtime.h>

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

constexpr int LD = TS + 1;  // padded LDS row length (elements)

// One 64x64 tile held across the 256 threads of a work-group: thread t keeps
// stored elements t, t + 256, ... (coalesced global loads).
template <class T>
struct TileRegs {
    T v[TE / 256];
};

template <class T>
__device__ __forceinline__ void fetch_tile(TileRegs<T> &r, const T *__restrict__ src) {
#pragma unroll
    for (int q = 0; q < TE / 256; ++q) r.v[q] = src[threadIdx.x + 256 * q];
}

// Stage into LDS as S[k][m] = op(tile)[m][k]  (A operand).
template <class T>
__device__ __forceinline__ void stage_A(T *S, const TileRegs<T> &r, bool trans) {
#pragma unroll
    for (int q = 0; q < TE / 256; ++q) {
        const int e = threadIdx.x + 256 * q;
        const int rr = e & (TS - 1), c = e >> 6;   // stored element (row rr, col c)
        if (!trans)
            S[c * LD + rr] = r.v[q];
        else
            S[rr * LD + c] = r.v[q];
    }
}

// Stage into LDS as S[k][n] = op(tile)[k][n]  (B operand).
template <class T>
__device__ __forceinline__ void stage_B(T *S, const TileRegs<T> &r, bool trans) {
#pragma unroll
    for (int q = 0; q < TE / 256; ++q) {
        const int e = threadIdx.x + 256 * q;
        const int rr = e & (TS - 1), c = e >> 6;
        if (!trans)
            S[rr * LD + c] = r.v[q];
        else
            S[c * LD + rr] = r.v[q];
    }
}

template <class T>
__device__ __forceinline__ void mfma_tile(const T *As, const T *Bs, typename Mfma<T>::acc_t acc[2][2],
                                          int lane, int wm, int wn) {
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll 4
    for (int kk = 0; kk < TS; kk += 4) {
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

// Tile contraction task.  The operands of pair p+1 are fetched into registers
// while the matrix cores work on pair p from LDS.
template <class T>
__global__ void __launch_bounds__(256) tile_gemm_kernel(T *__restrict__ arena,
                                                        const GemmTask *__restrict__ tasks,
                                                        const GemmPair *__restrict__ pairs, T *part,
                                                        int32_t *cnt) {
    __shared__ T As[TS * LD];
    __shared__ T Bs[TS * LD];
    __shared__ int32_t last;
    const GemmTask tk = tasks[blockIdx.x];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    typename Mfma<T>::acc_t acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = typename Mfma<T>::acc_t{0, 0, 0, 0};
    const bool ta = tk.flags & GF_TRANS_A, tb = tk.flags & GF_TRANS_B;
    TileRegs<T> ra, rb;
    if (tk.pair_count > 0) {
        const GemmPair pr = pairs[tk.pair_start];
        fetch_tile(ra, arena + pr.a_off);
        fetch_tile(rb, arena + pr.b_off);
    }
    for (int p = 0; p < tk.pair_count; ++p) {
        __syncthreads();
        stage_A(As, ra, ta);
        stage_B(Bs, rb, tb);
        __syncthreads();
        if (p + 1 < tk.pair_count) {
            const GemmPair pr = pairs[tk.pair_start + p + 1];
            fetch_tile(ra, arena + pr.a_off);
            fetch_tile(rb, arena + pr.b_off);
        }
        mfma_tile<T>(As, Bs, acc, lane, wm, wn);
    }
    if (tk.nchunk > 1) {
        // partial sums in accumulator order, reduced by the last arrival
        T *pp = part + tk.part_off + (int64_t)tk.chunk * TE;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int r = 0; r < 4; ++r) pp[((i * 2 + j) * 4 + r) * 256 + threadIdx.x] = acc[i][j][r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) last = atomicAdd(&cnt[tk.grp], 1) == tk.nchunk - 1;
        __syncthreads();
        if (!last) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = typename Mfma<T>::acc_t{0, 0, 0, 0};
        for (int c = 0; c < tk.nchunk; ++c) {
            const T *pc = part + tk.part_off + (int64_t)c * TE;
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j)
                    for (int r = 0; r < 4; ++r) acc[i][j][r] += pc[((i * 2 + j) * 4 + r) * 256 + threadIdx.x];
        }
        if (threadIdx.x == 0) atomicExch(&cnt[tk.grp], 0);
    }
    const int lr = lane & 15, lq = lane >> 4;
    const T alpha = (tk.flags & GF_NEGATE) ? T(-1) : T(1);
    T *C = arena + tk.c_off;
    const bool post = tk.flags & (GF_POST | GF_POST_RIGHT);
    if (tk.flags & GF_POST) {
        // C = alpha P S with S the accumulated sum: S becomes the B operand.
        __syncthreads();
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int r = 0; r < 4; ++r) {
                    const int m = wm + 16 * i + Mfma<T>::row(lq, r), n = wn + 16 * j + lr;
                    Bs[m * LD + n] = alpha * acc[i][j][r];
                    acc[i][j][r] = 0;
                }
        fetch_tile(ra, arena + tk.post_off);
        stage_A(As, ra, false);
        __syncthreads();
        mfma_tile<T>(As, Bs, acc, lane, wm, wn);
    } else if (tk.flags & GF_POST_RIGHT) {
        // C = ([C +] alpha S) P: the bracket becomes the A operand.
        const bool acc_c = tk.flags & GF_ACCUM;
        __syncthreads();
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int r = 0; r < 4; ++r) {
                    const int m = wm + 16 * i + Mfma<T>::row(lq, r), n = wn + 16 * j + lr;
                    T v = alpha * acc[i][j][r];
                    if (acc_c) v += C[n * TS + m];
                    As[n * LD + m] = v;
                    acc[i][j][r] = 0;
                }
        fetch_tile(rb, arena + tk.post_off);
        stage_B(Bs, rb, false);
        __syncthreads();
        mfma_tile<T>(As, Bs, acc, lane, wm, wn);
    }
    // stage the result column-major in LDS, then store coalesced
    __syncthreads();
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int r = 0; r < 4; ++r) {
                const int m = wm + 16 * i + Mfma<T>::row(lq, r), n = wn + 16 * j + lr;
                As[n * LD + m] = acc[i][j][r];
            }
    __syncthreads();
    const T a2 = post ? T(1) : alpha;
    const bool accum = (tk.flags & GF_ACCUM) && !post;
    const int t = threadIdx.x;
#pragma unroll 4
    for (int q = 0; q < TE / 256; ++q) {
        const int e = t + 256 * q;
        const int m = e & (TS - 1), n = e >> 6;
        const T v = a2 * As[n * LD + m];
        C[e] = accum ? C[e] + v : v;
    }
}

// Cholesky factor L and inverse W = L^-1 of one 64x64 tile, held in
// registers: lane r of wave q keeps row r of L and row r of V = W^T at the
// columns c = q + 4k (k < 16).  Step j uses the unscaled pivot d_j = L_jj:
// the owners of column j publish it (L and V) through LDS, then every thread
// subtracts L_rj L_cj / d_j from its entries of L and V_rj L_cj / d_j from V
// (forward elimination on the identity) for c > j, and the owners scale
// column j by 1/sqrt(d_j).  Entries above the diagonal of L are never read
// for the lower part and are masked on store.  One barrier per step
// (double-buffered columns); the published column is stored permuted
// (slot (c & 3) * 16 + c / 4) so a thread's 16 values are contiguous.  The
// 64 steps are unrolled at compile time so every register index is static.
template <class T, int J>
struct DiagStep {
    static __device__ __forceinline__ void run(T (&Lr)[16], T (&Vr)[16], T *colL, T *colV, int r, int q,
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
        const T inv_d = T(1) / d;
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
        if (q == qj) {
            const T sc = T(1) / sqrt(d);
            Lr[kj] *= sc;
            Vr[kj] *= sc;
        }
        DiagStep<T, J + 1>::run(Lr, Vr, colL, colV, r, q, bad);
    }
};
template <class T>
struct DiagStep<T, TS> {
    static __device__ __forceinline__ void run(T (&)[16], T (&)[16], T *, T *, int, int, bool &) {}
};

template <class T>
__global__ void __launch_bounds__(256) diag_kernel(T *__restrict__ A, T *__restrict__ Wa,
                                                   T *__restrict__ Wta,
                                                   const DiagTask *__restrict__ tasks,
                                                   int32_t *__restrict__ flag) {
    __shared__ T colL[2 * TS];
    __shared__ T colV[2 * TS];
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
    bool bad = false;
    DiagStep<T, 0>::run(Lr, Vr, colL, colV, r, q, bad);
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
    for (int e = t; e < TE; e += 256) {
        const int r = e & (TS - 1), c = e >> 6;
        S[r * LD + c] = s[e];
    }
    __syncthreads();
    T *d = dst + tk.dst_off;
    for (int e = t; e < TE; e += 256) {
        const int r = e & (TS - 1), c = e >> 6;   // dst(r, c) = src(c, r)
        d[e] = S[c * LD + r];
    }
}

// ---- tiled GEMV --------------------------------------------------------
template <class T>
struct Vec16;  // 16-byte load of consecutive tile elements, widened to double
template <>
struct Vec16<double> {
    static constexpr int R = 2;
    static __device__ __forceinline__ void load(const double *p, double *o) {
        const double2 v = *reinterpret_cast<const double2 *>(p);
        o[0] = v.x;
        o[1] = v.y;
    }
};
template <>
struct Vec16<float> {
    static constexpr int R = 4;
    static __device__ __forceinline__ void load(const float *p, double *o) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
};
template <>
struct Vec16<uint16_t> {   // bfloat16 storage
    static constexpr int R = 8;
    static __device__ __forceinline__ void load(const uint16_t *p, double *o) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = (double)__uint_as_float(w[i] << 16);
            o[2 * i + 1] = (double)__uint_as_float(w[i] & 0xffff0000u);
        }
    }
};

template <class T, int NW>
__global__ void __launch_bounds__(64 * NW) gemv_kernel(const T *__restrict__ arena, const double *__restrict__ x,
                                                       double *y, const GemvTask *__restrict__ tasks,
                                                       const GemvPair *__restrict__ pairs, const double *base,
                                                       double *part, int32_t *cnt) {
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
        part[tk.part_off + (int64_t)tk.chunk * TS + t] = s;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        int32_t old = 0;
        if (t == 0) old = atomicAdd(&cnt[tk.grp], 1);
        old = __shfl(old, 0, 64);
        if (old != tk.nchunk - 1) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s = 0.0;
        for (int c = 0; c < tk.nchunk; ++c) s += part[tk.part_off + (int64_t)c * TS + t];
        if (t == 0) atomicExch(&cnt[tk.grp], 0);
    }
    if (tk.base_off >= 0) s += base[tk.base_off + t];
    y[tk.y_off + t] = s;
}

// ---- launchers -----------------------------------------------------------
static inline unsigned grid_of(int64_t n) { return (unsigned)n; }

template <class T>
void launch_tile_gemm(T *arena, const GemmTask *tasks, const GemmPair *pairs, int64_t ntasks, hipStream_t s,
                      T *part, int32_t *cnt) {
    if (ntasks <= 0) return;
    hipLaunchKernelGGL(tile_gemm_kernel<T>, dim3(grid_of(ntasks)), dim3(256), 0, s, arena, tasks, pairs, part, cnt);
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
                 int64_t ntasks, hipStream_t s, const double *base, int32_t waves, double *part, int32_t *cnt) {
    if (ntasks <= 0) return;
    if (waves == 16)
        hipLaunchKernelGGL((gemv_kernel<T, 16>), dim3(grid_of(ntasks)), dim3(1024), 0, s, arena, x, y, tasks, pairs,
                           base, part, cnt);
    else
        hipLaunchKernelGGL((gemv_kernel<T, 4>), dim3(grid_of(ntasks)), dim3(256), 0, s, arena, x, y, tasks, pairs,
                           base, part, cnt);
}

template void launch_tile_gemm<double>(double *, const GemmTask *, const GemmPair *, int64_t, hipStream_t, double *,
                                       int32_t *);
template void launch_tile_gemm<float>(float *, const GemmTask *, const GemmPair *, int64_t, hipStream_t, float *,
                                      int32_t *);
template void launch_diag<double>(double *, double *, double *, const DiagTask *, int64_t, int32_t *, hipStream_t);
template void launch_diag<float>(float *, float *, float *, const DiagTask *, int64_t, int32_t *, hipStream_t);
template void launch_tile_transpose<double>(double *, double *, const CopyTask *, int64_t, hipStream_t);
template void launch_tile_transpose<float>(float *, float *, const CopyTask *, int64_t, hipStream_t);
template void launch_gemv<double>(const double *, const double *, double *, const GemvTask *, const GemvPair *,
                                  int64_t, hipStream_t, const double *, int32_t, double *, int32_t *);
template void launch_gemv<float>(const float *, const double *, double *, const GemvTask *, const GemvPair *,
                                 int64_t, hipStream_t, const double *, int32_t, double *, int32_t *);
template void launch_gemv<uint16_t>(const uint16_t *, const double *, double *, const GemvTask *,
                                    const GemvPair *, int64_t, hipStream_t, const double *, int32_t, double *,
                                    int32_t *);

}  // namespace hplmm
