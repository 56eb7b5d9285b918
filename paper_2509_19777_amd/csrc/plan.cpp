// Symbolic phase of libhplmm: validation, mortars (Sec. 3.3), the grouping
// W and reduction Q (Eqs. 20-21), the column layout of P (Eq. 23), contact
// grids (Eq. 26), device data layout and all launch task lists.
#include <algorithm>
#include <functional>
#include <array>
#include <map>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

#include "handle.h"

namespace hplmm {

namespace {

int64_t ceil_tiles(int64_t n) { return (n + TS - 1) / TS; }

// Gaussian mortar weights (Eq. 8) of one interface: H (N x nu) row-major.
std::vector<double> gaussian_weights(const std::vector<int32_t> &xyz, int32_t N, const std::vector<int32_t> &idx,
                                     double beta) {
    const int32_t nu = (int32_t)idx.size();
    std::vector<double> H((size_t)N * nu, 0.0);
    if (nu == 1) {
        std::fill(H.begin(), H.end(), 1.0);
        return H;
    }
    if (nu == N) {
        for (int32_t v = 0; v < N; ++v) H[(size_t)v * nu + v] = 1.0;
        return H;
    }
    auto d2 = [&](int32_t a, int32_t b) {
        const double dx = (double)(xyz[3 * a] - xyz[3 * b]), dy = (double)(xyz[3 * a + 1] - xyz[3 * b + 1]),
                     dz = (double)(xyz[3 * a + 2] - xyz[3 * b + 2]);
        return dx * dx + dy * dy + dz * dz;
    };
    std::vector<double> dmin((size_t)nu, INFINITY);
    for (int32_t i = 0; i < nu; ++i)
        for (int32_t j = 0; j < nu; ++j)
            if (i != j) dmin[(size_t)i] = std::min(dmin[(size_t)i], d2(idx[(size_t)i], idx[(size_t)j]));
    for (int32_t v = 0; v < N; ++v) {
        double s = 0.0;
        for (int32_t i = 0; i < nu; ++i) {
            const double a = std::exp(-d2(v, idx[(size_t)i]) / (beta * dmin[(size_t)i]));
            H[(size_t)v * nu + i] = a;
            s += a;
        }
        for (int32_t i = 0; i < nu; ++i) H[(size_t)v * nu + i] /= s;
    }
    return H;
}

// Append the factorisation program of a dense set: blocked right-looking
// Cholesky (diagonal tile, panel L_ik = A_ik L_kk^-T, trailing update) of the
// first nt_own tile columns (all of them for a full factorisation; a partial
// factorisation leaves the Schur complement in the trailing block), then the
// triangular inverse W = L^-1 of the factored block by diagonals, then its
// transposed tiles Wt = W^T.
// Algebraic mortar block of interface c (Eq. 9 in the algebraic form that
// follows Eq. 22): 3 Nc x 3 nu, row-major, rows 3 v + g (interface order),
// columns 3 i + g (mortar order).  Column (i, g) is 1 at dof g of mortar node
// i, 0 at the other mortar-node dofs, and -(A_FF)^-1 A_F,(i,g) on the free
// dofs F.  A_FF is factored by a banded Cholesky: interface nodes in
// ascending id order couple only to nearby positions.
std::vector<double> algebraic_block(const hplmm_system &sys, const int32_t *nodes, int32_t Nc, int32_t c,
                                    const std::vector<int32_t> &node_iface, const std::vector<int32_t> &node_irow,
                                    const std::vector<int32_t> &idx) {
    const int32_t n3 = 3 * Nc, k3 = 3 * (int32_t)idx.size();
    std::vector<int32_t> col((size_t)n3, -1), fpos((size_t)n3, -1), F;
    for (size_t i = 0; i < idx.size(); ++i)
        for (int g = 0; g < 3; ++g) col[(size_t)(3 * idx[i] + g)] = (int32_t)(3 * i + g);
    for (int32_t d = 0; d < n3; ++d)
        if (col[(size_t)d] < 0) {
            fpos[(size_t)d] = (int32_t)F.size();
            F.push_back(d);
        }
    const int64_t nf = (int64_t)F.size();
    std::vector<double> M((size_t)n3 * k3, 0.0);
    for (int32_t d = 0; d < n3; ++d)
        if (col[(size_t)d] >= 0) M[(size_t)d * k3 + col[(size_t)d]] = 1.0;
    if (nf == 0) return M;
    std::vector<double> L((size_t)(nf * nf), 0.0), B((size_t)(nf * k3), 0.0);
    int64_t bw = 0;
    for (int32_t v = 0; v < Nc; ++v) {
        const int32_t gv = nodes[v];
        for (int64_t p = sys.row_ptr[gv]; p < sys.row_ptr[gv + 1]; ++p) {
            const int32_t w = sys.col_idx[p];
            if (node_iface[(size_t)w] != c) continue;
            const int32_t lw = node_irow[(size_t)w];
            for (int gi = 0; gi < 3; ++gi) {
                const int64_t fr = fpos[(size_t)(3 * v + gi)];
                if (fr < 0) continue;   // constrained rows are dropped
                for (int di = 0; di < 3; ++di) {
                    const int32_t cd = 3 * lw + di;
                    const double a = sys.val[9 * p + 3 * gi + di];
                    if (fpos[(size_t)cd] >= 0) {
                        const int64_t fc = fpos[(size_t)cd];
                        L[(size_t)(fr * nf + fc)] = a;
                        bw = std::max<int64_t>(bw, fr > fc ? fr - fc : fc - fr);
                    } else {
                        B[(size_t)(fr * k3 + col[(size_t)cd])] = a;
                    }
                }
            }
        }
    }
    // A_FF = L L^T within the band (lower triangle of L, row-major)
    for (int64_t k = 0; k < nf; ++k) {
        double d = L[(size_t)(k * nf + k)];
        for (int64_t q = std::max<int64_t>(0, k - bw); q < k; ++q) d -= L[(size_t)(k * nf + q)] * L[(size_t)(k * nf + q)];
        if (!(d > 0.0)) fail(HPLMM_E_NOT_SPD, "algebraic mortars: interface block " + std::to_string(c) + " is not positive definite");
        const double lkk = std::sqrt(d);
        L[(size_t)(k * nf + k)] = lkk;
        for (int64_t i = k + 1; i <= std::min<int64_t>(nf - 1, k + bw); ++i) {
            double t = L[(size_t)(i * nf + k)];
            for (int64_t q = std::max<int64_t>(0, i - bw); q < k; ++q) t -= L[(size_t)(i * nf + q)] * L[(size_t)(k * nf + q)];
            L[(size_t)(i * nf + k)] = t / lkk;
        }
    }
    // A_FF X = A_FK by the two banded triangular solves; M_F = -X
    std::vector<double> x((size_t)nf);
    for (int32_t j = 0; j < k3; ++j) {
        for (int64_t i = 0; i < nf; ++i) {
            double t = B[(size_t)(i * k3 + j)];
            for (int64_t q = std::max<int64_t>(0, i - bw); q < i; ++q) t -= L[(size_t)(i * nf + q)] * x[(size_t)q];
            x[(size_t)i] = t / L[(size_t)(i * nf + i)];
        }
        for (int64_t i = nf - 1; i >= 0; --i) {
            double t = x[(size_t)i];
            for (int64_t q = i + 1; q <= std::min<int64_t>(nf - 1, i + bw); ++q) t -= L[(size_t)(q * nf + i)] * x[(size_t)q];
            x[(size_t)i] = t / L[(size_t)(i * nf + i)];
        }
        for (int64_t i = 0; i < nf; ++i) M[(size_t)F[(size_t)i] * k3 + j] = -x[(size_t)i];
    }
    return M;
}

// Tile envelope of a diagonal block of the fine matrix whose nodes are
// `nodes` (local node l = nodes[l], dofs 3l .. 3l+2): first[I] is the first
// tile column with a nonzero in tile row I (the padding rows past the block
// hold only their diagonal).  `loc` is a scratch map of every node to -1.
std::vector<int32_t> tile_envelope(const hplmm_system &sys, const int32_t *nodes, int64_t cnt,
                                   std::vector<int32_t> &loc) {
    for (int64_t l = 0; l < cnt; ++l) loc[(size_t)nodes[l]] = (int32_t)l;
    const int64_t nt = ceil_tiles(3 * cnt);
    std::vector<int32_t> first((size_t)nt);
    for (int64_t I = 0; I < nt; ++I) first[(size_t)I] = (int32_t)I;
    for (int64_t l = 0; l < cnt; ++l) {
        const int32_t v = nodes[l];
        int64_t lo = l;
        for (int64_t p = sys.row_ptr[v]; p < sys.row_ptr[v + 1]; ++p) {
            const int32_t u = loc[(size_t)sys.col_idx[p]];
            if (u >= 0) lo = std::min<int64_t>(lo, u);
        }
        const int32_t c = (int32_t)(3 * lo / TS);
        for (int64_t r = 3 * l; r < 3 * l + 3; ++r) first[(size_t)(r / TS)] = std::min(first[(size_t)(r / TS)], c);
    }
    for (int64_t l = 0; l < cnt; ++l) loc[(size_t)nodes[l]] = -1;
    return first;
}

// The factor program of a dense set.  With fuse_w the rows of W = L^-1 are
// formed in the Cholesky steps' launches; otherwise they go to ds.w_prog, one
// launch per row, to run after the factorisation (and beside other work).
// step_extra(k) may append tasks to step k's panel launch (they run after
// the diagonal tile k is factored).
void build_factor_program(DenseSet &ds, TaskLists &tl, int32_t set_id, std::vector<Launch> *out = nullptr,
                          const std::vector<int64_t> *ids = nullptr, bool fuse_w = true,
                          const std::function<void(int64_t)> &step_extra = {}) {
    std::vector<Launch> &prog = out ? *out : ds.factor_prog;
    if (!fuse_w) ds.w_prog.clear();
    const int64_t nm = (int64_t)ds.n.size();
    auto own = [&](int64_t m) { return ds.nt_own.empty() ? ds.nt[m] : ds.nt_own[m]; };
    int64_t maxk = 0;
    for (int64_t m = 0; m < nm; ++m) maxk = std::max(maxk, own(m));
    auto A = [&](int64_t m, int64_t I, int64_t J) { return ds.a_base + ds.rel[m] + tri_index(I, J) * TE; };
    // W = L^-1 exists for the factored rows only (I < own), so a partially
    // factored matrix may keep W and Wt in smaller slots of their own
    auto wrel = [&](int64_t m) { return ds.wrel.empty() ? ds.rel[m] : ds.wrel[m]; };
    auto W = [&](int64_t m, int64_t I, int64_t J) { return ds.w_base + wrel(m) + tri_index(I, J) * TE; };
    auto Wt = [&](int64_t m, int64_t I, int64_t J) {
        if (ds.wt_diag) {
            if (I != J) fail(HPLMM_E_ARG, "internal: off-diagonal Wt tile without storage");
            return ds.wt_base + ds.wdrel[m] + I * TE;
        }
        return ds.wt_base + wrel(m) + tri_index(I, J) * TE;
    };
    auto id = [&](int64_t m) { return (int32_t)(set_id * (1 << 26) + (ids ? (*ids)[m] : m)); };
    // first tile column of L's row I that can be nonzero (the envelope)
    auto first = [&](int64_t m, int64_t I) -> int64_t { return ds.first.empty() ? 0 : ds.first[m][I]; };
    auto push_pairs = [&](int64_t lo, int64_t hi, auto pair) {
        for (int64_t q = lo; q < hi; ++q) tl.pairs.push_back(pair(q));
        return (int32_t)std::max<int64_t>(0, hi - lo);
    };
    // row k of W = L^-1: W_kj = -W_kk sum_{q=j}^{k-1} L_kq W_qj, j < k, reading
    // rows of L and W finished before; an empty sum (row k uncoupled to earlier
    // rows) writes a zero tile
    // (with stored transposes the task also writes Wt_jk = W_kj^T)
    auto w_row = [&](int64_t m, int64_t k) {
        for (int64_t j = 0; j < k; ++j) {
            const int32_t ps = (int32_t)tl.pairs.size();
            const int32_t pc = push_pairs(std::max(j, first(m, k)), k, [&](int64_t q) {
                return GemmPair{A(m, k, q), W(m, q, j)};
            });
            GemmTask g{W(m, k, j), W(m, k, k), ps, pc, GF_POST | GF_NEGATE, 0};
            if (!ds.wt_diag) g.t_off = Wt(m, k, j);
            tl.gemm.push_back(g);
        }
    };
    // Left-looking tile Cholesky, two launches per step k: the diagonal tile
    // A_kk - sum_{p<k} L_kp L_kp^T is factored (the diagonal kernel subtracts
    // the last term, p = k - 1, itself), then the panel
    // L_ik = (A_ik - sum_p L_ip L_kp^T) L_kk^-T is formed in one task per tile.
    // Tiles left of a row's envelope are zero in A and stay zero in L: no
    // task writes them and no pair reads them.
    for (int64_t k = 0; k < maxk; ++k) {
        Launch d{LK_DIAG, (int64_t)tl.diag.size(), 0};
        for (int64_t m = 0; m < nm; ++m)
            if (own(m) > k)
                tl.diag.push_back({A(m, k, k), W(m, k, k), Wt(m, k, k), id(m), 0,
                                   k > 0 && first(m, k) < k ? A(m, k, k - 1) : -1});
        d.count = (int64_t)tl.diag.size() - d.start;
        prog.push_back(d);
        // the panel, in the same launch row k of W (fused) with the W_kk
        // just formed, and the terms p < k of the next diagonal tile's update
        Launch p{LK_GEMM, (int64_t)tl.gemm.size(), 0};
        for (int64_t m = 0; m < nm; ++m) {
            if (own(m) <= k) continue;
            for (int64_t i = k + 1; i < ds.nt[m]; ++i) {
                if (first(m, i) > k) continue;
                const int32_t ps = (int32_t)tl.pairs.size();
                const int32_t pc = push_pairs(std::max(first(m, i), first(m, k)), k, [&](int64_t q) {
                    return GemmPair{A(m, i, q), A(m, k, q)};
                });
                tl.gemm.push_back({A(m, i, k), Wt(m, k, k), ps, pc, GF_TRANS_B | GF_ACCUM | GF_NEGATE | GF_POST_RIGHT, 0});
            }
            if (fuse_w) w_row(m, k);
            if (k + 1 < own(m) && first(m, k + 1) < k) {
                const int32_t ps = (int32_t)tl.pairs.size();
                const int32_t pc = push_pairs(first(m, k + 1), k, [&](int64_t q) {
                    return GemmPair{A(m, k + 1, q), A(m, k + 1, q)};
                });
                tl.gemm.push_back({A(m, k + 1, k + 1), -1, ps, pc, GF_TRANS_B | GF_ACCUM | GF_NEGATE, 0});
            }
        }
        if (step_extra) step_extra(k);
        p.count = (int64_t)tl.gemm.size() - p.start;
        if (p.count) prog.push_back(p);
    }
    if (!fuse_w)
        for (int64_t k = 1; k < maxk; ++k) {
            Launch w{LK_GEMM, (int64_t)tl.gemm.size(), 0};
            for (int64_t m = 0; m < nm; ++m)
                if (own(m) > k) w_row(m, k);
            w.count = (int64_t)tl.gemm.size() - w.start;
            if (w.count) ds.w_prog.push_back(w);
        }
    // Partially factored matrices: Schur complement of the owned columns on
    // the remaining block, S_ij = A_ij - sum_{p < own} L_ip L_jp^T.
    {
        Launch u{LK_GEMM, (int64_t)tl.gemm.size(), 0};
        for (int64_t m = 0; m < nm; ++m) {
            const int64_t o = own(m);
            if (o == 0) continue;
            for (int64_t i = o; i < ds.nt[m]; ++i)
                for (int64_t j = o; j <= i; ++j) {
                    tl.gemm.push_back({A(m, i, j), -1, (int32_t)tl.pairs.size(), (int32_t)o,
                                       GF_TRANS_B | GF_ACCUM | GF_NEGATE, 0});
                    for (int64_t q = 0; q < o; ++q) tl.pairs.push_back({A(m, i, q), A(m, j, q)});
                }
        }
        u.count = (int64_t)tl.gemm.size() - u.start;
        if (u.count) prog.push_back(u);
    }
}

// Apply-time GEMV task lists y = W x and y = W^T x of a dense set.
void build_smoother_gemv(DenseSet &ds, std::vector<GemvTask> &vt, std::vector<GemvPair> &vp, int64_t w_abs,
                         int64_t wt_abs) {
    const int64_t nm = (int64_t)ds.n.size();
    ds.gemv_W.start = (int64_t)vt.size();
    // schedule the longest rows first
    std::vector<std::pair<int64_t, int64_t>> order;
    for (int64_t m = 0; m < nm; ++m)
        for (int64_t I = 0; I < ds.nt[m]; ++I) order.push_back({m, I});
    std::stable_sort(order.begin(), order.end(), [&](auto a, auto b) { return a.second > b.second; });
    for (auto [m, I] : order) {
        vt.push_back({ds.voff[m] + I * TS, (int32_t)vp.size(), (int32_t)(I + 1), -1});
        for (int64_t J = 0; J <= I; ++J) vp.push_back({w_abs + ds.rel[m] + tri_index(I, J) * TE, ds.voff[m] + J * TS});
    }
    ds.gemv_W.count = (int64_t)vt.size() - ds.gemv_W.start;
    std::stable_sort(order.begin(), order.end(), [&](auto a, auto b) {
        return (ds.nt[a.first] - a.second) > (ds.nt[b.first] - b.second);
    });
    ds.gemv_Wt.start = (int64_t)vt.size();
    for (auto [m, I] : order) {
        vt.push_back({ds.voff[m] + I * TS, (int32_t)vp.size(), (int32_t)(ds.nt[m] - I), -1});
        for (int64_t J = I; J < ds.nt[m]; ++J)
            vp.push_back({wt_abs + ds.rel[m] + tri_index(J, I) * TE, ds.voff[m] + J * TS});
    }
    ds.gemv_Wt.count = (int64_t)vt.size() - ds.gemv_Wt.start;
}

// S = W^T W for every matrix of a dense set (the inverse smoother form): lower
// tiles S_ij = sum_{k >= i} W_ki^T W_kj, i >= j, one task per tile, W as both
// operands (the left one read transposed).  FP64: W and S in the FP64 arena.
// Reduced precision (low): the rounded W at low_w_base, S written to
// low_s_base of the FP32 arena.
void build_inverse_program(DenseSet &ds, TaskLists &tl, bool low) {
    const int64_t wb = low ? ds.low_w_base : ds.w_base, sb = low ? ds.low_s_base : ds.s_base;
    auto W = [&](int64_t m, int64_t I, int64_t J) { return wb + ds.rel[m] + tri_index(I, J) * TE; };
    auto S = [&](int64_t m, int64_t I, int64_t J) { return sb + ds.rel[m] + tri_index(I, J) * TE; };
    Launch L{LK_GEMM, (int64_t)tl.gemm.size(), 0};
    for (int64_t m = 0; m < (int64_t)ds.n.size(); ++m)
        for (int64_t i = 0; i < ds.nt[m]; ++i)
            for (int64_t j = 0; j <= i; ++j) {
                tl.gemm.push_back({S(m, i, j), -1, (int32_t)tl.pairs.size(), (int32_t)(ds.nt[m] - i),
                                   (int32_t)GF_TRANS_A, 0});
                for (int64_t k = i; k < ds.nt[m]; ++k) tl.pairs.push_back({W(m, k, i), W(m, k, j)});
            }
    L.count = (int64_t)tl.gemm.size() - L.start;
    if (L.count) ds.inverse_prog.push_back(L);
}

// Apply-time lists of y = S x (inverse form): one task per tile row I, longest
// rows first, with pairs S_IJ, J <= I; pair J < I also yields row J's part
// S_IJ^T x_I, kept in a slot of the partial buffer.  The slots of row J (from
// rows I = J+1 .. nt-1) lie contiguously, and one sum task per row adds them.
void build_sym_gemv(DenseSet &ds, std::vector<GemvTask> &vt, std::vector<SymPair> &sp, std::vector<SymReduce> &rt,
                    int64_t &part_len, int64_t s_abs) {
    const int64_t nm = (int64_t)ds.n.size();
    std::vector<int64_t> pbase((size_t)nm);
    for (int64_t m = 0; m < nm; ++m) {
        pbase[(size_t)m] = part_len;
        part_len += ds.nt[m] * (ds.nt[m] - 1) / 2 * TS;
    }
    auto slot = [&](int64_t m, int64_t I, int64_t J) {   // row J's part from row I > J
        const int64_t row = J * (ds.nt[m] - 1) - J * (J - 1) / 2;
        return pbase[(size_t)m] + (row + I - J - 1) * TS;
    };
    std::vector<std::pair<int64_t, int64_t>> order;
    for (int64_t m = 0; m < nm; ++m)
        for (int64_t I = 0; I < ds.nt[m]; ++I) order.push_back({m, I});
    std::stable_sort(order.begin(), order.end(), [&](auto a, auto b) { return a.second > b.second; });
    ds.gemv_S.start = (int64_t)vt.size();
    auto valid = [&](int64_t m, int64_t I) { return (int32_t)std::min<int64_t>(TS, ds.n[m] - I * TS); };
    for (auto [m, I] : order) {
        vt.push_back({ds.voff[m] + I * TS, (int32_t)sp.size(), (int32_t)(I + 1), -1});
        for (int64_t J = 0; J <= I; ++J)
            sp.push_back({s_abs + ds.rel[m] + tri_index(I, J) * TE, ds.voff[m] + J * TS, J < I ? slot(m, I, J) : -1,
                          valid(m, I), valid(m, J)});
    }
    ds.gemv_S.count = (int64_t)vt.size() - ds.gemv_S.start;
    ds.gemv_S.sym = true;
    ds.red_S.start = (int64_t)rt.size();
    for (int64_t m = 0; m < nm; ++m)
        for (int64_t J = 0; J + 1 < ds.nt[m]; ++J)
            rt.push_back({ds.voff[m] + J * TS, slot(m, J + 1, J), (int32_t)(ds.nt[m] - 1 - J), 0});
    ds.red_S.count = (int64_t)rt.size() - ds.red_S.start;
}

// Bytes of a sum launch: the slots read, y read and written.
double sym_reduce_bytes(const std::vector<SymReduce> &rt, Range r) {
    double b = 0.0;
    for (int64_t i = r.start; i < r.start + r.count; ++i) b += ((double)rt[(size_t)i].count + 2.0) * TS * 8.0;
    return b;
}

// Algorithmic bytes of a GEMV launch: every tile and x segment read, y written.
double gemv_bytes(const std::vector<GemvTask> &vt, Range r, double elem) {
    double b = 0.0;
    for (int64_t i = r.start; i < r.start + r.count; ++i)
        b += (double)vt[(size_t)i].pair_count * (TE * elem + TS * 8.0) + TS * 8.0;
    return b;
}

// Bytes the symmetric GEMV launch reads and writes: the valid part of every
// tile (the lower triangle of the diagonal one), its x segment and the row's
// own x segment, the row of y and a slot per transposed product.
double sym_gemv_bytes(const std::vector<GemvTask> &vt, const std::vector<SymPair> &sp, Range r, double elem) {
    double b = 0.0;
    for (int64_t i = r.start; i < r.start + r.count; ++i) {
        const GemvTask &t = vt[(size_t)i];
        for (int32_t q = 0; q < t.pair_count; ++q) {
            const SymPair &pr = sp[(size_t)(t.pair_start + q)];
            // off the diagonal the valid block; on it the lower triangle
            const double e = pr.p_off >= 0 ? (double)pr.rows * pr.cols : 0.5 * pr.rows * (pr.rows + 1.0);
            b += e * elem + TS * 8.0 + (pr.p_off >= 0 ? TS * 8.0 : 0.0);
        }
        b += 2.0 * TS * 8.0;
    }
    return b;
}

// Re-emit the rows of GEMV launch r at the end of vt so that the launch
// spreads over about target work-groups (a work-group streams tiles at a small
// fraction of the device bandwidth): rows longer than the chunk length (at
// least 4 pairs) are cut into chunks whose partial sums a reduction launch
// after the product adds in chunk order.  target 0 returns r unchanged.
// part_len grows to what the launch needs.
Range split_rows(std::vector<GemvTask> &vt, Range r, int64_t target, int64_t &part_len) {
    if (target <= 0) return r;
    int64_t total = 0;
    for (int64_t i = r.start; i < r.start + r.count; ++i) total += vt[(size_t)i].pair_count;
    const int64_t chunk = std::max<int64_t>(4, (total + target - 1) / target);
    const int64_t start = (int64_t)vt.size();
    int64_t part = 0;
    bool any = false;
    for (int64_t i = r.start; i < r.start + r.count; ++i) {
        const GemvTask t = vt[(size_t)i];
        const int64_t nc = (t.pair_count + chunk - 1) / chunk;
        if (nc <= 1) {
            vt.push_back(t);
            continue;
        }
        if (nc > 32767) fail(HPLMM_E_ARG, "internal: GEMV row too long to split");
        const int64_t per = (t.pair_count + nc - 1) / nc;
        for (int64_t c = 0; c < nc; ++c) {
            GemvTask u = t;
            u.pair_start = (int32_t)(t.pair_start + c * per);
            u.pair_count = (int32_t)std::min<int64_t>(per, t.pair_count - c * per);
            u.part_off = part;
            u.chunk = (int16_t)c;
            u.nchunk = (int16_t)nc;
            vt.push_back(u);
        }
        part += nc * TS;
        any = true;
    }
    Range out = r;
    out.start = start;
    out.count = (int64_t)vt.size() - start;
    out.split = any;
    part_len = std::max(part_len, part);
    return out;
}

// The shapes of one coarse-sweep launch: by default a launch with fewer than
// 128 rows is split over about 256 work-groups and a larger one is left alone;
// the autotuner may also pick the unsplit rows or 256 to 2048 work-groups.
GemvShapes sweep_shapes(std::vector<GemvTask> &vt, Range base, int64_t &part_len) {
    GemvShapes g;
    const int32_t def = base.count < 128 ? 256 : 0;
    const double bytes = gemv_bytes(vt, base, 8.0);   // the same rows whatever the shape
    for (int32_t t : {def, 0, 256, 512, 1024, 2048}) {
        if (!g.target.empty() && t == def) continue;
        g.target.push_back(t);
        g.var.push_back(split_rows(vt, base, t, part_len));
        g.var.back().bytes = bytes;
    }
    return g;
}

}  // namespace

// Split the long sums of a GEMM launch that has too few tasks to fill the
// device: a work-group loads its tile pairs at a small fraction of the device
// bandwidth, so a chain of k products is cut into about sqrt(k/2)-pair
// chunks that run on different compute units; a finishing pass after the
// launch adds each task's partials in order and applies its epilogue.
void split_program(std::vector<Launch> &prog, TaskLists &tl) {
    for (Launch &L : prog) {
        if (L.kind != LK_GEMM || L.count >= 256) continue;
        int64_t total = 0;
        for (int64_t i = L.start; i < L.start + L.count; ++i) total += tl.gemm[(size_t)i].pair_count;
        const int64_t floor_per = std::max<int64_t>(2, (total + 511) / 512);   // at most ~512 work-groups
        const int64_t start = (int64_t)tl.gemm.size();
        int64_t part = 0;
        bool any = false;
        for (int64_t i = L.start; i < L.start + L.count; ++i) {
            const GemmTask t = tl.gemm[(size_t)i];
            const int64_t k = t.pair_count;
            const int64_t per = std::max<int64_t>(floor_per, (int64_t)std::lround(std::sqrt((double)k / 2.0)));
            const int64_t nc = k >= 4 ? (k + per - 1) / per : 1;
            if (nc <= 1) {
                tl.gemm.push_back(t);
                continue;
            }
            any = true;
            const int64_t each = (k + nc - 1) / nc;
            for (int64_t c = 0; c < nc; ++c) {
                GemmTask u = t;
                u.pair_start = (int32_t)(t.pair_start + c * each);
                u.pair_count = (int32_t)std::min<int64_t>(each, k - c * each);
                u.part_off = part;
                u.chunk = (int16_t)c;
                u.nchunk = (int16_t)nc;
                tl.gemm.push_back(u);
            }
            part += nc * TE;
        }
        if (!any) {
            tl.gemm.resize((size_t)start);
            continue;
        }
        L.start = start;
        L.count = (int64_t)tl.gemm.size() - start;
        L.split = true;
        tl.part_len = std::max(tl.part_len, part);
    }
}

// Algorithmic flops of every GEMM launch: 2*64^3 per tile product.
void fill_flops(std::vector<Launch> &prog, const TaskLists &tl) {
    for (Launch &L : prog) {
        if (L.kind != LK_GEMM) continue;
        double f = 0.0;
        for (int64_t i = L.start; i < L.start + L.count; ++i) {
            const GemmTask &t = tl.gemm[(size_t)i];
            f += (double)t.pair_count + ((t.flags & (GF_POST | GF_POST_RIGHT)) && t.chunk == 0 ? 1.0 : 0.0);
        }
        L.flops = f * 2.0 * TS * TS * TS;
    }
}

namespace {

void layout_set(DenseSet &ds) {
    ds.rel.resize(ds.n.size());
    ds.nt.resize(ds.n.size());
    ds.voff.resize(ds.n.size());
    int64_t off = 0, vo = 0;
    for (size_t m = 0; m < ds.n.size(); ++m) {
        ds.nt[m] = ceil_tiles(ds.n[m]);
        ds.rel[m] = off;
        off += tri_tiles(ds.nt[m]) * TE;
        ds.voff[m] = vo;
        vo += ds.nt[m] * TS;
    }
    ds.region = off;
    ds.vec_len = vo;
}

void pad_ones(const DenseSet &ds, std::vector<int64_t> &out, int64_t a_base) {
    for (size_t m = 0; m < ds.n.size(); ++m)
        for (int64_t r = ds.n[m]; r < ds.nt[m] * TS; ++r)
            out.push_back(a_base + ds.rel[m] + tri_index(r / TS, r / TS) * TE + (r % TS) * TS + (r % TS));
}


// ---- multifrontal coarse factorisation: symbolic phase ----------------------------
// Nested dissection of the interface graph (two interfaces are adjacent when
// the coarse operator couples them) by recursive coordinate bisection of the
// interface centroids; each bisection's separator is the boundary layer of
// the side with fewer dofs.  Subsets of at most leaf_dofs dofs become leaves.
struct NDCtx {
    const std::vector<std::vector<int32_t>> &adj;
    const std::vector<std::array<double, 3>> &cen;
    const std::vector<int32_t> &dofs;
    CoarseMF &mf;
    std::vector<int32_t> mark;
    int64_t leaf_dofs;
};

int32_t nd_build(NDCtx &x, std::vector<int32_t> I, int32_t par, int32_t side, int32_t depth) {
    CoarseMF &mf = x.mf;
    const int32_t t = mf.n_fronts++;
    mf.parent.push_back(par);
    mf.side.push_back(side);
    mf.level.push_back(depth);
    mf.own.emplace_back();
    mf.bnd.emplace_back();
    int64_t tot = 0;
    for (int32_t c : I) tot += x.dofs[(size_t)c];
    if (tot <= x.leaf_dofs || I.size() <= 2) {
        std::sort(I.begin(), I.end());
        mf.own[(size_t)t] = I;
        return t;
    }
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t c : I)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], x.cen[(size_t)c][d]);
            hi[d] = std::max(hi[d], x.cen[(size_t)c][d]);
        }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
        if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    std::stable_sort(I.begin(), I.end(), [&](int32_t a, int32_t b) {
        if (x.cen[(size_t)a][ax] != x.cen[(size_t)b][ax]) return x.cen[(size_t)a][ax] < x.cen[(size_t)b][ax];
        return a < b;
    });
    const size_t half = I.size() / 2;
    std::vector<int32_t> L(I.begin(), I.begin() + (long)half), R(I.begin() + (long)half, I.end());
    // mark: 1 = left, 2 = right
    for (int32_t c : L) x.mark[(size_t)c] = 1;
    for (int32_t c : R) x.mark[(size_t)c] = 2;
    std::vector<int32_t> sepL, sepR;
    int64_t dL = 0, dR = 0;
    for (int32_t c : L)
        for (int32_t e : x.adj[(size_t)c])
            if (x.mark[(size_t)e] == 2) {
                sepL.push_back(c);
                dL += x.dofs[(size_t)c];
                break;
            }
    for (int32_t c : R)
        for (int32_t e : x.adj[(size_t)c])
            if (x.mark[(size_t)e] == 1) {
                sepR.push_back(c);
                dR += x.dofs[(size_t)c];
                break;
            }
    for (int32_t c : I) x.mark[(size_t)c] = 0;
    std::vector<int32_t> sep = dL <= dR ? sepL : sepR;
    std::vector<int32_t> &from = dL <= dR ? L : R;
    for (int32_t c : sep) x.mark[(size_t)c] = 3;
    from.erase(std::remove_if(from.begin(), from.end(), [&](int32_t c) { return x.mark[(size_t)c] == 3; }), from.end());
    for (int32_t c : sep) x.mark[(size_t)c] = 0;
    std::sort(sep.begin(), sep.end());
    mf.own[(size_t)t] = sep;
    if (!L.empty()) nd_build(x, L, t, 0, depth + 1);
    if (!R.empty()) nd_build(x, R, t, 1, depth + 1);
    return t;
}

void build_coarse_mf(Handle &h, const hplmm_system &sys, const hplmm_partition &part,
                     const std::vector<int32_t> &iface_nu, const std::vector<int64_t> &iface_moff,
                     std::vector<CoarsePair> &pairs, int64_t &off64) {
    CoarseMF &mf = h.mf;
    const int32_t nI = part.n_ifaces;
    if (h.n_mortar == 0 || nI == 0) return;
    std::vector<std::vector<int32_t>> adj((size_t)nI);
    for (const auto &pr : pairs)
        if (pr.c != pr.c2) {
            adj[(size_t)pr.c].push_back(pr.c2);
            adj[(size_t)pr.c2].push_back(pr.c);
        }
    for (auto &a : adj) {
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
    }
    std::vector<std::array<double, 3>> cen((size_t)nI);
    std::vector<int32_t> dofs((size_t)nI);
    for (int32_t c = 0; c < nI; ++c) {
        double s[3] = {0, 0, 0};
        const int64_t p0 = part.iface_ptr[c], p1 = part.iface_ptr[c + 1];
        for (int64_t q = p0; q < p1; ++q)
            for (int d = 0; d < 3; ++d) s[d] += sys.node_xyz[3 * (int64_t)part.iface_nodes[q] + d];
        for (int d = 0; d < 3; ++d) cen[(size_t)c][d] = s[d] / (double)(p1 - p0);
        dofs[(size_t)c] = 3 * iface_nu[(size_t)c];
    }
    NDCtx x{adj, cen, dofs, mf, std::vector<int32_t>((size_t)nI, 0), h.coarse_leaf_dofs};
    std::vector<int32_t> all((size_t)nI);
    std::iota(all.begin(), all.end(), 0);
    nd_build(x, all, -1, 0, 0);
    const int32_t nf = mf.n_fronts;
    // children lists
    std::vector<std::array<int32_t, 2>> child((size_t)nf, {-1, -1});
    for (int32_t t = 0; t < nf; ++t)
        if (mf.parent[(size_t)t] >= 0) child[(size_t)mf.parent[(size_t)t]][(size_t)mf.side[(size_t)t]] = t;
    // owners
    mf.iface_front.assign((size_t)nI, -1);
    for (int32_t t = 0; t < nf; ++t)
        for (int32_t c : mf.own[(size_t)t]) mf.iface_front[(size_t)c] = t;
    for (int32_t c = 0; c < nI; ++c)
        if (mf.iface_front[(size_t)c] < 0) fail(HPLMM_E_ARG, "internal: interface missing from the dissection");
    // symbolic boundaries in postorder (children have larger ids than parents,
    // so decreasing ids visit every child before its parent)
    std::vector<uint8_t> elim((size_t)nI, 0);
    std::vector<int32_t> stamp((size_t)nI, -1);
    for (int32_t t = nf - 1; t >= 0; --t) {
        std::vector<int32_t> cand;
        for (int32_t c : mf.own[(size_t)t]) stamp[(size_t)c] = t;
        auto consider = [&](int32_t e) {
            if (elim[(size_t)e] || stamp[(size_t)e] == t) return;
            stamp[(size_t)e] = t;
            cand.push_back(e);
        };
        for (int32_t c : mf.own[(size_t)t])
            for (int32_t e : adj[(size_t)c]) consider(e);
        for (int s = 0; s < 2; ++s)
            if (child[(size_t)t][s] >= 0)
                for (int32_t e : mf.bnd[(size_t)child[(size_t)t][s]]) consider(e);
        std::sort(cand.begin(), cand.end());
        mf.bnd[(size_t)t] = cand;
        for (int32_t c : mf.own[(size_t)t]) elim[(size_t)c] = 1;
    }
    if (!mf.bnd[0].empty()) fail(HPLMM_E_ARG, "internal: root front has a boundary");
    // sizes, positions, storage
    mf.d.resize(nf);
    mf.u.resize(nf);
    mf.nt_d.resize(nf);
    mf.nt_u.resize(nf);
    mf.rel.resize(nf);
    mf.wrel.resize(nf);
    mf.ltrel.resize(nf);
    mf.voff.resize(nf);
    mf.iface_pos.assign((size_t)nI, -1);
    std::vector<std::unordered_map<int32_t, int64_t>> pos((size_t)nf);
    int64_t off = 0, wo = 0, lt = 0, vo = 0;
    for (int32_t t = 0; t < nf; ++t) {
        int64_t d = 0, u = 0;
        for (int32_t c : mf.own[(size_t)t]) {
            pos[(size_t)t][c] = d;
            mf.iface_pos[(size_t)c] = d;
            d += dofs[(size_t)c];
        }
        const int64_t ntd = ceil_tiles(d);
        for (int32_t c : mf.bnd[(size_t)t]) {
            pos[(size_t)t][c] = ntd * TS + u;
            u += dofs[(size_t)c];
        }
        const int64_t ntu = ceil_tiles(u);
        mf.d[(size_t)t] = d;
        mf.u[(size_t)t] = u;
        mf.nt_d[(size_t)t] = ntd;
        mf.nt_u[(size_t)t] = ntu;
        mf.rel[(size_t)t] = off;
        off += tri_tiles(ntd + ntu) * TE;
        mf.wrel[(size_t)t] = wo;
        wo += tri_tiles(ntd) * TE;
        mf.ltrel[(size_t)t] = lt;
        lt += ntd * ntu * TE;
        mf.voff[(size_t)t] = vo;
        vo += (ntd + ntu) * TS;
    }
    mf.region = off;
    mf.w_region = wo;
    mf.lt_region = lt;
    mf.vec_len = vo;
    mf.a_base = off64;
    off64 += off;
    mf.w_base = off64;
    off64 += wo;
    mf.wt_base = off64;
    off64 += wo;
    mf.lt_base = off64;
    off64 += lt;
    mf.ng_base = off64;
    off64 += lt;
    int32_t nl = 0;
    for (int32_t t = 0; t < nf; ++t) nl = std::max(nl, mf.level[(size_t)t] + 1);
    mf.n_levels = nl;
    std::vector<std::vector<int32_t>> at((size_t)nl);
    for (int32_t t = 0; t < nf; ++t) at[(size_t)mf.level[(size_t)t]].push_back(t);
    // extend-add maps: child boundary dof -> parent front position
    std::vector<int64_t> map_off((size_t)nf, -1);
    for (int32_t t = 0; t < nf; ++t) {
        const int32_t par = mf.parent[(size_t)t];
        if (par < 0) continue;
        map_off[(size_t)t] = (int64_t)mf.maps.size();
        for (int32_t c : mf.bnd[(size_t)t]) {
            auto it = pos[(size_t)par].find(c);
            if (it == pos[(size_t)par].end()) fail(HPLMM_E_ARG, "internal: boundary interface missing from the parent front");
            for (int32_t j = 0; j < dofs[(size_t)c]; ++j) mf.maps.push_back((int32_t)(it->second + j));
        }
    }
    // and their inverses over the parent's positions
    std::vector<int64_t> inv_off((size_t)nf, -1);
    for (int32_t t = 0; t < nf; ++t) {
        const int32_t par = mf.parent[(size_t)t];
        if (par < 0) continue;
        inv_off[(size_t)t] = (int64_t)mf.inv.size();
        mf.inv.resize(mf.inv.size() + (size_t)((mf.nt_d[(size_t)par] + mf.nt_u[(size_t)par]) * TS), -1);
        for (int64_t rr = 0; rr < mf.u[(size_t)t]; ++rr) {
            const int64_t p = mf.maps[(size_t)(map_off[(size_t)t] + rr)];
            if (p < 0 || p >= (mf.nt_d[(size_t)par] + mf.nt_u[(size_t)par]) * TS ||
                mf.inv[(size_t)(inv_off[(size_t)t] + p)] != -1)
                fail(HPLMM_E_ARG, "internal plan check failed: extend-add map");
            mf.inv[(size_t)(inv_off[(size_t)t] + p)] = (int32_t)rr;
        }
    }
    mf.inv_at = inv_off;
    auto A = [&](int32_t t, int64_t I, int64_t J) { return mf.a_base + mf.rel[(size_t)t] + tri_index(I, J) * TE; };
    auto W = [&](int32_t t, int64_t I, int64_t J) { return mf.w_base + mf.wrel[(size_t)t] + tri_index(I, J) * TE; };
    auto Wt = [&](int32_t t, int64_t I, int64_t J) { return mf.wt_base + mf.wrel[(size_t)t] + tri_index(I, J) * TE; };
    // G = L21 W11 (boundary rows times the inverse of the own block) is stored
    // negated, NG(I, J) with I a boundary tile and J an own tile, and as
    // per-tile transposes NGT(I, J) = NG(I, J)^T.
    auto NGT = [&](int32_t t, int64_t I, int64_t J) {
        return mf.lt_base + mf.ltrel[(size_t)t] + (I * mf.nt_d[(size_t)t] + J) * TE;
    };
    auto NG = [&](int32_t t, int64_t I, int64_t J) {
        return mf.ng_base + mf.ltrel[(size_t)t] + (I * mf.nt_d[(size_t)t] + J) * TE;
    };
    mf.factor_prog.assign((size_t)nl, {});
    mf.ext_lvl.assign((size_t)nl, Range{});
    mf.vec_ext.assign((size_t)nl, Range{});
    mf.bwd_copy.assign((size_t)nl, Range{});
    mf.fwd.assign((size_t)nl, Range{});
    mf.bwd.assign((size_t)nl, Range{});
    mf.fwd_shapes.assign((size_t)nl, GemvShapes{});
    mf.bwd_shapes.assign((size_t)nl, GemvShapes{});
    mf.va_ptr.push_back(0);
    for (int32_t l = 0; l < nl; ++l) {
        // factorisation of this level's fronts
        DenseSet lv;
        std::vector<int64_t> ids;
        for (int32_t t : at[(size_t)l]) {
            lv.n.push_back(mf.d[(size_t)t] + mf.u[(size_t)t]);
            lv.nt.push_back(mf.nt_d[(size_t)t] + mf.nt_u[(size_t)t]);
            lv.nt_own.push_back(mf.nt_d[(size_t)t]);
            lv.rel.push_back(mf.rel[(size_t)t]);
            lv.wrel.push_back(mf.wrel[(size_t)t]);
            ids.push_back(t);
        }
        lv.a_base = mf.a_base;
        lv.w_base = mf.w_base;
        lv.wt_base = mf.wt_base;
        build_factor_program(lv, h.tl64, 2, &mf.factor_prog[(size_t)l], &ids);
        // NG = -L21 W11, each task also writing its transpose NGT
        Launch g{LK_GEMM, (int64_t)h.tl64.gemm.size(), 0};
        for (int32_t t : at[(size_t)l]) {
            const int64_t nd = mf.nt_d[(size_t)t];
            for (int64_t I = 0; I < mf.nt_u[(size_t)t]; ++I)
                for (int64_t J = 0; J < nd; ++J) {
                    GemmTask task{NG(t, I, J), -1, (int32_t)h.tl64.pairs.size(), (int32_t)(nd - J), GF_NEGATE, 0};
                    task.t_off = NGT(t, I, J);
                    h.tl64.gemm.push_back(task);
                    for (int64_t K = J; K < nd; ++K) h.tl64.pairs.push_back({A(t, nd + I, K), W(t, K, J)});
                }
        }
        g.count = (int64_t)h.tl64.gemm.size() - g.start;
        if (g.count) mf.factor_prog[(size_t)l].push_back(g);
        // extend-add of the children (level l+1) into this level's fronts:
        // the parent tiles (PI, PJ) with rows of one child in both PI and PJ
        {
            Range r{(int64_t)mf.ext.size(), 0};
            for (int32_t t : at[(size_t)l]) {
                const int64_t ntp = mf.nt_d[(size_t)t] + mf.nt_u[(size_t)t];
                std::vector<char> hit[2];
                for (int s = 0; s < 2; ++s) {
                    const int32_t ch = child[(size_t)t][s];
                    if (ch < 0) continue;
                    hit[s].assign((size_t)ntp, 0);
                    for (int64_t rr = 0; rr < mf.u[(size_t)ch]; ++rr)
                        hit[s][(size_t)(mf.maps[(size_t)(map_off[(size_t)ch] + rr)] / TS)] = 1;
                }
                for (int64_t I = 0; I < ntp; ++I)
                    for (int64_t J = 0; J <= I; ++J) {
                        ExtendTile e{A(t, I, J), {-1, -1}, {-1, -1}, {0, 0}, (int32_t)I, (int32_t)J, (int32_t)ntp, 0};
                        bool any = false;
                        for (int s = 0; s < 2; ++s) {
                            const int32_t ch = child[(size_t)t][s];
                            if (ch < 0 || !hit[s][(size_t)I] || !hit[s][(size_t)J]) continue;
                            e.child_off[s] = mf.a_base + mf.rel[(size_t)ch];
                            e.inv_off[s] = inv_off[(size_t)ch];
                            e.nt_d[s] = (int32_t)mf.nt_d[(size_t)ch];
                            any = true;
                        }
                        if (any) mf.ext.push_back(e);
                    }
            }
            r.count = (int64_t)mf.ext.size() - r.start;
            mf.ext_lvl[(size_t)l] = r;
        }
        // forward vector extend-add: parent slot <- sum of child boundary slots
        {
            Range r{(int64_t)mf.va_dst.size(), 0};
            for (int32_t t : at[(size_t)l]) {
                std::map<int64_t, std::vector<int64_t>> src;
                for (int s = 0; s < 2; ++s) {
                    const int32_t ch = child[(size_t)t][s];
                    if (ch < 0) continue;
                    for (int64_t rr = 0; rr < mf.u[(size_t)ch]; ++rr)
                        src[mf.maps[(size_t)(map_off[(size_t)ch] + rr)]].push_back(
                            mf.voff[(size_t)ch] + mf.nt_d[(size_t)ch] * TS + rr);
                }
                for (auto &kv : src) {
                    mf.va_dst.push_back(mf.voff[(size_t)t] + kv.first);
                    for (int64_t q : kv.second) mf.va_src.push_back(q);
                    mf.va_ptr.push_back((int64_t)mf.va_src.size());
                }
            }
            r.count = (int64_t)mf.va_dst.size() - r.start;
            mf.vec_ext[(size_t)l] = r;
        }
        // backward: this level's boundary values from the parent front
        {
            Range r{(int64_t)mf.cp_dst.size(), 0};
            for (int32_t t : at[(size_t)l]) {
                const int32_t par = mf.parent[(size_t)t];
                if (par < 0) continue;
                for (int64_t rr = 0; rr < mf.u[(size_t)t]; ++rr) {
                    mf.cp_dst.push_back(mf.voff[(size_t)t] + mf.nt_d[(size_t)t] * TS + rr);
                    mf.cp_src.push_back(mf.voff[(size_t)par] + mf.maps[(size_t)(map_off[(size_t)t] + rr)]);
                }
            }
            r.count = (int64_t)mf.cp_dst.size() - r.start;
            mf.bwd_copy[(size_t)l] = r;
        }
        // GEMV lists of the solve
        auto &vt = h.vtasks;
        auto &vp = h.vpairs;
        // The front vectors live in one buffer: w (right-hand side, updated in
        // place on the boundary) at 0, y at vec_len, x at 2 vec_len.
        const int64_t vw = 0, vy = mf.vec_len, vx = 2 * mf.vec_len;
        // forward: y_d = W11 w_d and w_u += NG w_d in one launch
        mf.fwd[(size_t)l].start = (int64_t)vt.size();
        for (int32_t t : at[(size_t)l]) {
            const int64_t nd = mf.nt_d[(size_t)t], o = mf.voff[(size_t)t];
            for (int64_t I = 0; I < nd; ++I) {
                vt.push_back({vy + o + I * TS, (int32_t)vp.size(), (int32_t)(I + 1), -1});
                for (int64_t J = 0; J <= I; ++J) vp.push_back({W(t, I, J), vw + o + J * TS});
            }
            if (nd == 0) continue;
            for (int64_t I = 0; I < mf.nt_u[(size_t)t]; ++I) {
                vt.push_back({vw + o + (nd + I) * TS, (int32_t)vp.size(), (int32_t)nd, vw + o + (nd + I) * TS});
                for (int64_t J = 0; J < nd; ++J) vp.push_back({NG(t, I, J), vw + o + J * TS});
            }
        }
        mf.fwd[(size_t)l].count = (int64_t)vt.size() - mf.fwd[(size_t)l].start;
        // backward: x_d = W11^T y_d + NG^T x_u in one launch
        mf.bwd[(size_t)l].start = (int64_t)vt.size();
        for (int32_t t : at[(size_t)l]) {
            const int64_t nd = mf.nt_d[(size_t)t], nu = mf.nt_u[(size_t)t], o = mf.voff[(size_t)t];
            for (int64_t I = 0; I < nd; ++I) {
                vt.push_back({vx + o + I * TS, (int32_t)vp.size(), (int32_t)(nd - I + nu), -1});
                for (int64_t J = I; J < nd; ++J) vp.push_back({Wt(t, J, I), vy + o + J * TS});
                for (int64_t K = 0; K < nu; ++K) vp.push_back({NGT(t, K, I), vx + o + (nd + K) * TS});
            }
        }
        mf.bwd[(size_t)l].count = (int64_t)vt.size() - mf.bwd[(size_t)l].start;
        mf.fwd_shapes[(size_t)l] = sweep_shapes(vt, mf.fwd[(size_t)l], h.gemv_part_len);
        mf.bwd_shapes[(size_t)l] = sweep_shapes(vt, mf.bwd[(size_t)l], h.gemv_part_len);
        mf.fwd[(size_t)l] = mf.fwd_shapes[(size_t)l].var[0];
        mf.bwd[(size_t)l] = mf.bwd_shapes[(size_t)l].var[0];
    }
    // right-hand side in, solution out
    mf.init_map.assign((size_t)mf.vec_len, -1);
    for (int32_t c = 0; c < nI; ++c) {
        const int32_t t = mf.iface_front[(size_t)c];
        for (int32_t j = 0; j < dofs[(size_t)c]; ++j) {
            const int64_t slot = mf.voff[(size_t)t] + mf.iface_pos[(size_t)c] + j;
            mf.init_map[(size_t)slot] = iface_moff[(size_t)c] + j;
            mf.out_dst.push_back(iface_moff[(size_t)c] + j);
            mf.out_src.push_back(slot);
        }
    }
    for (int32_t t = 0; t < nf; ++t)
        for (int64_t r = mf.d[(size_t)t]; r < mf.nt_d[(size_t)t] * TS; ++r)
            mf.pad_ones.push_back(A(t, r / TS, r / TS) + (r % TS) * TS + (r % TS));
    // the coarse Galerkin pairs go to the front that eliminates the earlier interface
    int64_t voffp = 0;
    for (auto &pr : pairs) {
        int32_t t1 = mf.iface_front[(size_t)pr.c], t2 = mf.iface_front[(size_t)pr.c2];
        int32_t t = t1;
        if (t1 != t2) {
            // the deeper front must have the other interface on its boundary
            t = mf.level[(size_t)t1] >= mf.level[(size_t)t2] ? t1 : t2;
        }
        auto i1 = pos[(size_t)t].find(pr.c), i2 = pos[(size_t)t].find(pr.c2);
        if (i1 == pos[(size_t)t].end() || i2 == pos[(size_t)t].end())
            fail(HPLMM_E_ARG, "internal: coarse coupling outside its front");
        pr.f_off = mf.a_base + mf.rel[(size_t)t];
        pr.pos1 = (int32_t)i1->second;
        pr.pos2 = (int32_t)i2->second;
        pr.v_off = voffp;
        voffp += 9 * (int64_t)iface_nu[(size_t)pr.c] * iface_nu[(size_t)pr.c2];
    }
    h.n_pair_vals = voffp;
    for (int32_t l = 0; l < nl; ++l) split_program(mf.factor_prog[(size_t)l], h.tl64);
    for (int32_t l = 0; l < nl; ++l) fill_flops(mf.factor_prog[(size_t)l], h.tl64);
    for (int32_t l = 0; l < nl; ++l)
        for (const Launch &L : mf.factor_prog[(size_t)l]) mf.flops += L.flops;
    for (int32_t t = 0; t < nf; ++t) {
        const double dd = (double)mf.d[(size_t)t], uu = (double)mf.u[(size_t)t];
        mf.factor_bytes += 8.0 * (dd * (dd + 1) / 2 + dd * uu);
    }
}
}  // namespace

// The method's own set-up flops and application bytes from the unpadded
// sizes (grain interiors N with k mortar and c = k + 1 or k columns, contact
// grids n, coarse fronts with d own and u boundary dofs), and the flops the
// set-up's tile tasks issue, for comparison.
static void method_work(Handle &h) {
    const bool inv = h.smoother_form == HPLMM_SMOOTHER_INVERSE;
    // stored element: FP64, FP32 or bfloat16 W in the factor form; S in FP64
    // or (reduced precision) FP32 in the inverse form
    const double se = h.smoother_precision == 64 ? 8.0 : (inv || h.smoother_precision == 32 ? 4.0 : 2.0);
    double fg = 0.0, fc = 0.0, ff = 0.0, bs = 0.0, bb = 0.0;
    for (size_t m = 0; m < h.gset.n.size(); ++m) {
        const double N = (double)h.gset.n[m], k = (double)h.gm_k[m], c = (double)h.gm_ncol[m];
        fg += N * N * N / 3.0 + 2.0 * N * N * c + 2.0 * N * k * k;
        // smoother: S (one triangle) or W and W^T (two passes over one triangle);
        // x read and y written
        bs += (inv ? 1.0 : 2.0) * se * N * (N + 1) / 2 + 16.0 * N;
        // restriction and prolongation: the N x c block twice, vectors in and out
        bb += 2.0 * (8.0 * N * c + 8.0 * (N + c));
    }
    for (size_t m = 0; m < h.cset.n.size(); ++m) {
        const double n = (double)h.cset.n[m];
        fc += n * n * n / 3.0;
        bs += (inv ? 1.0 : 2.0) * se * n * (n + 1) / 2 + 16.0 * n;
    }
    double bf = 0.0;
    for (int32_t t = 0; t < h.mf.n_fronts; ++t) {
        const double d = (double)h.mf.d[(size_t)t], u = (double)h.mf.u[(size_t)t];
        ff += d * d * d / 3.0 + d * d * u + d * u * u;
        bf += 2.0 * (8.0 * (d * (d + 1) / 2 + d * u) + 8.0 * (2.0 * d + 2.0 * u));
    }
    h.method_setup_flops[0] = fg;
    h.method_setup_flops[1] = fc;
    h.method_setup_flops[2] = ff;
    h.method_setup_flops[3] = fg + fc + ff;
    auto sum = [](const std::vector<Launch> &prog) {
        double f = 0.0;
        for (const Launch &L : prog) f += L.flops;
        return f;
    };
    h.issued_setup_flops[0] =
        sum(h.gset.factor_prog) + sum(h.gset.w_prog) + sum(h.gset.inverse_prog) + sum(h.basis_prog) +
        sum(h.basis_x_prog);
    h.issued_setup_flops[1] = sum(h.cset.factor_prog) + sum(h.cset.inverse_prog);
    h.issued_setup_flops[2] = h.mf.flops;
    h.issued_setup_flops[3] = h.issued_setup_flops[0] + h.issued_setup_flops[1] + h.issued_setup_flops[2];
    const double n = (double)h.N;
    // two residual products r - A z, each reading r and z and writing the result
    const double sp = 2.0 * (h.spmv_bytes + 24.0 * (double)h.n_nodes);
    h.method_apply_bytes[0] = bs;
    h.method_apply_bytes[1] = bb;
    h.method_apply_bytes[2] = bf;
    h.method_apply_bytes[3] = sp;
    // plus the vector traffic between the steps: gathers into the local
    // vectors, the combines of Eqs. 16 and 25 (read and write of N-vectors)
    h.method_apply_bytes[4] = bs + bb + bf + sp + 8.0 * 6.0 * n;
}

// Basis tasks (Eqs. 23-24) of the grain matrices ms, appended to tl and prog:
// BP_Y: Y = W R; BP_X: X = W^T Y written over R; BP_K: K = Y^T Y;
// BP_XT: per-tile transposes of X into the XT region.
void append_basis_program(Handle &h, TaskLists &tl, const std::vector<int64_t> &ms, std::vector<Launch> &prog,
                          int parts) {
    auto Wg = [&](int64_t m, int64_t I, int64_t J) { return h.gset.w_base + h.gset.rel[m] + tri_index(I, J) * TE; };
    auto Rt = [&](int64_t base, int64_t m, int64_t I, int64_t C) { return base + (C * h.gset.nt[m] + I) * TE; };
    if (parts & BP_Y) {
        Launch L1{LK_GEMM, (int64_t)tl.gemm.size(), 0};
        for (int64_t m : ms)
            for (int64_t C = 0; C < h.gm_ntc[(size_t)m]; ++C)
                for (int64_t I = 0; I < h.gset.nt[m]; ++I) {
                    tl.gemm.push_back({Rt(h.gm_ytoff[(size_t)m], m, I, C), -1, (int32_t)tl.pairs.size(), (int32_t)(I + 1), 0, 0});
                    for (int64_t J = 0; J <= I; ++J) tl.pairs.push_back({Wg(m, I, J), Rt(h.gm_roff[(size_t)m], m, J, C)});
                }
        L1.count = (int64_t)tl.gemm.size() - L1.start;
        if (L1.count) prog.push_back(L1);
    }
    if (parts & BP_X) {
        Launch L2{LK_GEMM, (int64_t)tl.gemm.size(), 0};
        // X_IC = sum_{J >= I} W_JI^T Y_JC: W read transposed
        for (int64_t m : ms)
            for (int64_t C = 0; C < h.gm_ntc[(size_t)m]; ++C)
                for (int64_t I = 0; I < h.gset.nt[m]; ++I) {
                    tl.gemm.push_back({Rt(h.gm_roff[(size_t)m], m, I, C), -1, (int32_t)tl.pairs.size(),
                                       (int32_t)(h.gset.nt[m] - I), GF_TRANS_A, 0});
                    for (int64_t J = I; J < h.gset.nt[m]; ++J)
                        tl.pairs.push_back({Wg(m, J, I), Rt(h.gm_ytoff[(size_t)m], m, J, C)});
                }
        L2.count = (int64_t)tl.gemm.size() - L2.start;
        if (L2.count) prog.push_back(L2);
    }
    if (parts & BP_K) {
        Launch L3{LK_GEMM, (int64_t)tl.gemm.size(), 0};
        for (int64_t m : ms)
            for (int64_t C1 = 0; C1 < h.gm_ntc[(size_t)m]; ++C1)
                for (int64_t C2 = 0; C2 <= C1; ++C2) {
                    tl.gemm.push_back({h.gm_koff[(size_t)m] + tri_index(C1, C2) * TE, -1, (int32_t)tl.pairs.size(),
                                       (int32_t)h.gset.nt[m], GF_TRANS_A, 0});
                    for (int64_t I = 0; I < h.gset.nt[m]; ++I)
                        tl.pairs.push_back({Rt(h.gm_ytoff[(size_t)m], m, I, C1), Rt(h.gm_ytoff[(size_t)m], m, I, C2)});
                }
        L3.count = (int64_t)tl.gemm.size() - L3.start;
        if (L3.count) prog.push_back(L3);
    }
    if (parts & BP_XT) {
        Launch L4{LK_TRANSPOSE, (int64_t)tl.copy.size(), 0};
        for (int64_t m : ms)
            for (int64_t C = 0; C < h.gm_ntc[(size_t)m]; ++C)
                for (int64_t I = 0; I < h.gset.nt[m]; ++I)
                    tl.copy.push_back({Rt(h.gm_roff[(size_t)m], m, I, C),
                                       h.gm_xtoff[(size_t)m] + (I * h.gm_ntc[(size_t)m] + C) * TE});
        L4.count = (int64_t)tl.copy.size() - L4.start;
        if (L4.count) prog.push_back(L4);
    }
}

void build_plan(Handle &h, const hplmm_system &sys_in, const hplmm_partition &part, const hplmm_mortar &mort,
                const hplmm_options &opt, hipStream_t s, bool dry_run) {
    const int64_t n = sys_in.n_nodes;
    if (n <= 0 || !sys_in.row_ptr || !sys_in.col_idx || !sys_in.val || !sys_in.node_xyz)
        fail(HPLMM_E_ARG, "system arrays missing");
    // constrained dofs (Eq. 2's Dirichlet rows beyond the eliminated clamp):
    // the plan works on a copy of the matrix whose constrained rows and
    // columns are those of the identity and of the load with zeros there
    std::vector<double> cval, crhs;
    hplmm_system sys = sys_in;
    h.n_fixed = 0;
    if (sys_in.dof_fixed) {
        const int64_t nnzb = sys_in.row_ptr[n];
        if (sys_in.row_ptr[0] != 0 || nnzb < 0) fail(HPLMM_E_ARG, "row_ptr must start at 0");
        cval.assign(sys_in.val, sys_in.val + 9 * nnzb);
        for (int64_t v = 0; v < n; ++v)
            for (int64_t p = sys_in.row_ptr[v]; p < sys_in.row_ptr[v + 1]; ++p) {
                const int64_t w = sys_in.col_idx[p];
                if (w < 0 || w >= n) fail(HPLMM_E_ARG, "column index out of range");
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        const bool fa = sys_in.dof_fixed[3 * v + a] != 0, fb = sys_in.dof_fixed[3 * w + b] != 0;
                        if (fa || fb) cval[(size_t)(9 * p + 3 * a + b)] = (v == w && a == b) ? 1.0 : 0.0;
                    }
            }
        for (int64_t d = 0; d < 3 * n; ++d) h.n_fixed += sys_in.dof_fixed[d] != 0;
        sys.val = cval.data();
        if (sys_in.rhs) {
            crhs.assign(sys_in.rhs, sys_in.rhs + 3 * n);
            for (int64_t d = 0; d < 3 * n; ++d)
                if (sys_in.dof_fixed[d]) crhs[(size_t)d] = 0.0;
            sys.rhs = crhs.data();
        }
        sys.dof_fixed = nullptr;
    }
    if (!part.node_grain || part.n_grains < 0 || part.n_ifaces < 0 || (part.n_ifaces > 0 && (!part.iface_ptr || !part.iface_nodes)))
        fail(HPLMM_E_ARG, "partition arrays missing");
    if (part.n_nodes != n) fail(HPLMM_E_ARG, "partition and system disagree on n_nodes");
    if (part.n_contacts < 0 || (part.n_contacts > 0 && (!part.contact_ptr || !part.contact_nodes)))
        fail(HPLMM_E_ARG, "contact arrays missing");
    if (mort.n <= 0 || !(mort.beta > 0)) fail(HPLMM_E_ARG, "mortar n must be > 0 and beta > 0");
    if (mort.kind != HPLMM_MORTAR_GAUSSIAN && mort.kind != HPLMM_MORTAR_ALGEBRAIC)
        fail(HPLMM_E_ARG, "unknown mortar kind");
    h.mortar_kind = mort.kind;
    if (opt.smoother_precision != 64 && opt.smoother_precision != 32 && opt.smoother_precision != 16)
        fail(HPLMM_E_ARG, "smoother_precision must be 64, 32 or 16");
    h.smoother_precision = opt.smoother_precision;
    if (opt.smoother_form < HPLMM_SMOOTHER_AUTO || opt.smoother_form > HPLMM_SMOOTHER_INVERSE)
        fail(HPLMM_E_ARG, "smoother_form must be 0 (auto), 1 (factors) or 2 (inverse)");
    // auto: the inverse form (at reduced precision its S is the Gram matrix of
    // the rounded W, definite however coarse the rounding)
    h.smoother_form = opt.smoother_form != HPLMM_SMOOTHER_AUTO ? opt.smoother_form : HPLMM_SMOOTHER_INVERSE;
    if (opt.coarse_leaf_dofs < 0) fail(HPLMM_E_ARG, "coarse_leaf_dofs must be >= 0");
    h.coarse_leaf_dofs = opt.coarse_leaf_dofs > 0 ? opt.coarse_leaf_dofs : 192;
    h.n_nodes = n;
    h.N = 3 * n;
    h.nnzb = sys.row_ptr[n];
    if (sys.row_ptr[0] != 0) fail(HPLMM_E_ARG, "row_ptr[0] must be 0");
    for (int64_t v = 0; v < n; ++v) {
        if (sys.row_ptr[v + 1] < sys.row_ptr[v]) fail(HPLMM_E_ARG, "row_ptr not monotone");
        for (int64_t p = sys.row_ptr[v]; p < sys.row_ptr[v + 1]; ++p) {
            const int32_t w = sys.col_idx[p];
            if (w < 0 || w >= n) fail(HPLMM_E_ARG, "column index out of range");
            if (p > sys.row_ptr[v] && sys.col_idx[p - 1] >= w) fail(HPLMM_E_ARG, "columns not strictly ascending");
            // symmetric pattern
            const int32_t *b0 = sys.col_idx + sys.row_ptr[w], *b1 = sys.col_idx + sys.row_ptr[w + 1];
            if (!std::binary_search(b0, b1, (int32_t)v)) fail(HPLMM_E_ARG, "sparsity pattern not symmetric");
        }
    }
    h.n_grains = part.n_grains;
    h.n_ifaces = part.n_ifaces;
    h.n_contacts = part.n_contacts;
    // ---- classification (W, Eq. 20) ---------------------------------------
    std::vector<int32_t> node_iface((size_t)n, -1), node_irow((size_t)n, -1);
    for (int32_t c = 0; c < part.n_ifaces; ++c) {
        if (part.iface_ptr[c + 1] <= part.iface_ptr[c]) fail(HPLMM_E_PARTITION, "empty interface");
        for (int64_t p = part.iface_ptr[c]; p < part.iface_ptr[c + 1]; ++p) {
            const int32_t v = part.iface_nodes[p];
            if (v < 0 || v >= n) fail(HPLMM_E_PARTITION, "interface node out of range");
            if (node_iface[(size_t)v] >= 0) fail(HPLMM_E_PARTITION, "node in two interfaces");
            node_iface[(size_t)v] = c;
            node_irow[(size_t)v] = (int32_t)(p - part.iface_ptr[c]);
        }
    }
    for (int64_t v = 0; v < n; ++v) {
        const int32_t g = part.node_grain[v];
        if (g >= part.n_grains || g < -1) fail(HPLMM_E_PARTITION, "grain id out of range");
        if ((g >= 0) == (node_iface[(size_t)v] >= 0))
            fail(HPLMM_E_PARTITION, "every node must be interior to one grain or on one interface");
    }
    for (int64_t v = 0; v < n; ++v)
        for (int64_t p = sys.row_ptr[v]; p < sys.row_ptr[v + 1]; ++p) {
            const int32_t gv = part.node_grain[v], gw = part.node_grain[sys.col_idx[p]];
            if (gv >= 0 && gw >= 0 && gv != gw) fail(HPLMM_E_PARTITION, "A couples the interiors of two grains");
        }
    // ---- mortars (Eqs. 7-8) and Q ------------------------------------------
    std::vector<int32_t> iface_nu((size_t)part.n_ifaces);
    std::vector<int64_t> iface_moff((size_t)part.n_ifaces), iface_hoff((size_t)part.n_ifaces);
    h.h_H.clear();
    h.h_mortar_idx.clear();
    int64_t moff = 0;
    for (int32_t c = 0; c < part.n_ifaces; ++c) {
        const int64_t p0 = part.iface_ptr[c];
        const int32_t Nc = (int32_t)(part.iface_ptr[c + 1] - p0);
        std::vector<int32_t> xyz((size_t)Nc * 3);
        for (int32_t v = 0; v < Nc; ++v)
            for (int d = 0; d < 3; ++d) xyz[(size_t)3 * v + d] = sys.node_xyz[3 * (int64_t)part.iface_nodes[p0 + v] + d];
        auto idx = place_mortars(xyz.data(), Nc, mort.n);
        auto H = mort.kind == HPLMM_MORTAR_GAUSSIAN
                     ? gaussian_weights(xyz, Nc, idx, mort.beta)
                     : algebraic_block(sys, part.iface_nodes + p0, Nc, c, node_iface, node_irow, idx);
        iface_nu[(size_t)c] = (int32_t)idx.size();
        iface_moff[(size_t)c] = moff;
        iface_hoff[(size_t)c] = (int64_t)h.h_H.size();
        moff += 3 * (int64_t)idx.size();
        h.h_H.insert(h.h_H.end(), H.begin(), H.end());
        h.h_mortar_idx.insert(h.h_mortar_idx.end(), idx.begin(), idx.end());
    }
    h.h_iface_hoff = iface_hoff;
    h.n_mortar = moff;
    // ---- grain matrices and the columns of P (Eq. 23) -----------------------
    std::vector<std::vector<int32_t>> gnodes((size_t)part.n_grains);
    for (int64_t v = 0; v < n; ++v)
        if (part.node_grain[v] >= 0) gnodes[(size_t)part.node_grain[v]].push_back((int32_t)v);
    std::vector<int32_t> grain_mat((size_t)part.n_grains, -1);
    std::vector<int32_t> node_gmat((size_t)n, -1), node_local((size_t)n, -1);
    for (int32_t g = 0; g < part.n_grains; ++g) {
        if (gnodes[(size_t)g].empty()) continue;
        grain_mat[(size_t)g] = (int32_t)h.gm_grain.size();
        h.gm_grain.push_back(g);
    }
    const int64_t nG = (int64_t)h.gm_grain.size();
    for (int64_t m = 0; m < nG; ++m) {
        auto &nodes = gnodes[(size_t)h.gm_grain[(size_t)m]];
        for (size_t l = 0; l < nodes.size(); ++l) {
            node_gmat[(size_t)nodes[l]] = (int32_t)m;
            node_local[(size_t)nodes[l]] = (int32_t)l;
        }
        h.gset.n.push_back(3 * (int64_t)nodes.size());
    }
    for (int32_t c = 0; c < part.n_ifaces; ++c)
        for (int64_t p = part.iface_ptr[c]; p < part.iface_ptr[c + 1]; ++p)
            node_local[(size_t)part.iface_nodes[p]] = (int32_t)(p - part.iface_ptr[c]);
    // interfaces coupled to each grain's interior (nonzero columns of Abar_gi)
    std::vector<std::vector<int32_t>> gadj((size_t)nG);
    std::vector<AbarWork> abar;
    {
        std::vector<int32_t> seen;
        for (int64_t v = 0; v < n; ++v) {
            const int32_t m = node_gmat[(size_t)v];
            if (m < 0) continue;
            seen.clear();
            for (int64_t p = sys.row_ptr[v]; p < sys.row_ptr[v + 1]; ++p) {
                const int32_t c = node_iface[(size_t)sys.col_idx[p]];
                if (c >= 0 && std::find(seen.begin(), seen.end(), c) == seen.end()) seen.push_back(c);
            }
            std::sort(seen.begin(), seen.end());
            for (int32_t c : seen) {
                gadj[(size_t)m].push_back(c);
                abar.push_back({(int32_t)v, c, (int32_t)m, node_local[(size_t)v], 0, 0});
            }
        }
    }
    std::vector<std::unordered_map<int32_t, int32_t>> lcol((size_t)nG);
    h.gm_k.resize(nG);
    h.gm_corr.assign(nG, -1);
    h.gm_ncol.resize(nG);
    h.gm_ntc.resize(nG);
    h.h_corr_grains.clear();
    for (int64_t m = 0; m < nG; ++m) {
        auto &a = gadj[(size_t)m];
        std::sort(a.begin(), a.end());
        a.erase(std::unique(a.begin(), a.end()), a.end());
        int32_t k = 0;
        for (int32_t c : a) {
            lcol[(size_t)m][c] = k;
            k += 3 * iface_nu[(size_t)c];
        }
        h.gm_k[(size_t)m] = k;
        bool loaded = false;
        if (sys.rhs)
            for (int32_t v : gnodes[(size_t)h.gm_grain[(size_t)m]])
                for (int d = 0; d < 3; ++d) loaded |= sys.rhs[3 * (int64_t)v + d] != 0.0;
        if (loaded) {
            h.gm_corr[(size_t)m] = (int32_t)h.h_corr_grains.size();
            h.h_corr_grains.push_back(h.gm_grain[(size_t)m]);
        }
        h.gm_ncol[(size_t)m] = k + (loaded ? 1 : 0);
        h.gm_ntc[(size_t)m] = (int32_t)ceil_tiles(h.gm_ncol[(size_t)m]);
    }
    for (auto &w : abar) w.lcol0 = lcol[(size_t)w.m][w.c];
    // what the learned-basis surrogate reads: lattice coordinates, per-node
    // operator features, grain node lists and grain-interface adjacency
    {
        h.sg_xyz.assign(sys.node_xyz, sys.node_xyz + 3 * n);
        h.sg_logtr.assign((size_t)n, 0.f);
        h.sg_fill.assign((size_t)n, 0.f);
        for (int64_t v = 0; v < n; ++v) {
            double tr = 0.0;
            for (int64_t p = sys.row_ptr[v]; p < sys.row_ptr[v + 1]; ++p)
                if (sys.col_idx[p] == v) tr = sys.val[9 * p] + sys.val[9 * p + 4] + sys.val[9 * p + 8];
            h.sg_logtr[(size_t)v] = tr > 0.0 ? (float)std::log(tr) : 0.f;
            h.sg_fill[(size_t)v] = (float)(sys.row_ptr[v + 1] - sys.row_ptr[v]) / 27.f;
        }
        h.sg_gnodes_ptr.assign(1, 0);
        h.sg_gnodes.clear();
        h.sg_adj_ptr.assign(1, 0);
        h.sg_adj.clear();
        h.sg_lcol.clear();
        for (int64_t m = 0; m < nG; ++m) {
            for (int32_t v : gnodes[(size_t)h.gm_grain[(size_t)m]]) h.sg_gnodes.push_back(v);
            h.sg_gnodes_ptr.push_back((int64_t)h.sg_gnodes.size());
            for (int32_t c : gadj[(size_t)m]) {
                h.sg_adj.push_back(c);
                h.sg_lcol.push_back(lcol[(size_t)m][c]);
            }
            h.sg_adj_ptr.push_back((int64_t)h.sg_adj.size());
        }
        h.sg_iface_nu = iface_nu;
        h.sg_iface_ptr.assign(part.iface_ptr, part.iface_ptr + part.n_ifaces + 1);
        h.sg_iface_nodes.assign(part.iface_nodes, part.iface_nodes + (part.n_ifaces ? part.iface_ptr[part.n_ifaces] : 0));
    }
    h.n_corr = (int64_t)h.h_corr_grains.size();
    h.n_coarse = h.n_mortar + h.n_corr;
    // ---- contact grids (Eq. 26) -----------------------------------------------
    std::vector<int64_t> cn_cnt((size_t)n + 1, 0);
    for (int32_t c = 0; c < part.n_contacts; ++c) {
        if (part.contact_ptr[c + 1] <= part.contact_ptr[c]) fail(HPLMM_E_PARTITION, "empty contact grid");
        for (int64_t p = part.contact_ptr[c]; p < part.contact_ptr[c + 1]; ++p) {
            const int32_t v = part.contact_nodes[p];
            if (v < 0 || v >= n) fail(HPLMM_E_PARTITION, "contact node out of range");
            if (p > part.contact_ptr[c] && part.contact_nodes[p - 1] >= v)
                fail(HPLMM_E_PARTITION, "contact nodes must be strictly ascending");
            cn_cnt[(size_t)v + 1]++;
        }
        h.cset.n.push_back(3 * (part.contact_ptr[c + 1] - part.contact_ptr[c]));
    }
    // ---- tile envelopes of the grain and contact-grid blocks ---------------------
    {
        std::vector<int32_t> loc((size_t)n, -1);
        h.gset.first.resize((size_t)nG);
        for (int64_t m = 0; m < nG; ++m) {
            const auto &nodes = gnodes[(size_t)h.gm_grain[(size_t)m]];
            h.gset.first[(size_t)m] = tile_envelope(sys, nodes.data(), (int64_t)nodes.size(), loc);
        }
        h.cset.first.resize((size_t)part.n_contacts);
        for (int32_t c = 0; c < part.n_contacts; ++c)
            h.cset.first[(size_t)c] = tile_envelope(sys, part.contact_nodes + part.contact_ptr[c],
                                                    part.contact_ptr[c + 1] - part.contact_ptr[c], loc);
    }
    // ---- layout ------------------------------------------------------------------
    layout_set(h.gset);
    layout_set(h.cset);
    int64_t off64 = 0, off32 = 0, offbf = 0;
    auto take64 = [&](int64_t k) { const int64_t o = off64; off64 += k; return o; };
    const bool lowp = h.smoother_precision != 64;
    const bool inverse = h.smoother_form == HPLMM_SMOOTHER_INVERSE;
    // the inverse form reads W transposed in its products: of Wt it keeps only
    // the diagonal tiles that the Cholesky panels multiply by
    auto wt_elems = [&](DenseSet &ds) {
        ds.wt_diag = inverse;
        if (!inverse) return ds.region;
        ds.wdrel.resize(ds.n.size());
        int64_t o = 0;
        for (size_t m = 0; m < ds.n.size(); ++m) {
            ds.wdrel[m] = o;
            o += ds.nt[m] * TE;
        }
        return o;
    };
    // the basis by substitution with the sparse factor (inverse form), which
    // leaves W = L^-1 to the grain inverse alone
    h.basis_subst = inverse;
    h.negi_off = h.basis_subst ? take64(TE) : -1;
    h.gset.a_base = take64(h.gset.region);
    h.gset.w_base = take64(h.gset.region);
    h.gset.wt_base = take64(wt_elems(h.gset));
    h.gm_roff.resize(nG);
    h.gm_ytoff.resize(nG);
    h.gm_xtoff.resize(nG);
    h.gm_koff.resize(nG);
    h.gm_coff.resize(nG);
    int64_t r_region = 0, k_region = 0;
    for (int64_t m = 0; m < nG; ++m) {
        r_region += h.gset.nt[m] * h.gm_ntc[(size_t)m] * TE;
        k_region += tri_tiles(h.gm_ntc[(size_t)m]) * TE;
    }
    const int64_t r_base = take64(r_region), y_base = take64(r_region), xt_base = take64(r_region),
                  k_base = take64(k_region);
    {
        int64_t ro = 0, ko = 0, co = 0;
        for (int64_t m = 0; m < nG; ++m) {
            h.gm_roff[(size_t)m] = r_base + ro;
            h.gm_ytoff[(size_t)m] = y_base + ro;
            h.gm_xtoff[(size_t)m] = xt_base + ro;
            ro += h.gset.nt[m] * h.gm_ntc[(size_t)m] * TE;
            h.gm_koff[(size_t)m] = k_base + ko;
            ko += tri_tiles(h.gm_ntc[(size_t)m]) * TE;
            h.gm_coff[(size_t)m] = co;
            co += h.gm_ntc[(size_t)m] * TS;
        }
        h.gcol_len = co;
    }
    // contact grids factored in FP32: the reduced-precision factor form only
    const bool c32 = lowp && !inverse;
    if (!c32) {
        h.cset.a_base = take64(h.cset.region);
        h.cset.w_base = take64(h.cset.region);
        h.cset.wt_base = take64(wt_elems(h.cset));
    } else {
        h.c_stage_base = take64(h.cset.region);
        h.cset.a_base = off32;
        off32 += h.cset.region;
        h.cset.w_base = off32;
        off32 += h.cset.region;
        h.cset.wt_base = off32;
        off32 += h.cset.region;
    }
    // reduced-precision smoother copies.  Inverse form: W of both sets rounded
    // to the storage precision (FP32 arena at 32, bfloat16 arena at 16) and
    // S = Wp^T Wp formed from it, kept in FP32.  Factor form: W and Wt.
    if (inverse && lowp) {
        for (DenseSet *ds : {&h.gset, &h.cset}) {
            if (h.smoother_precision == 32) {
                ds->low_w_base = off32;
                off32 += ds->region;
            } else {
                ds->low_w_base = offbf;
                offbf += ds->region;
            }
            ds->low_s_base = off32;
            off32 += ds->region;
        }
    } else if (h.smoother_precision == 32) {
        h.gset.low_w_base = off32;
        off32 += h.gset.region;
        h.gset.low_wt_base = off32;
        off32 += h.gset.region;
        h.cset.low_w_base = h.cset.w_base;
        h.cset.low_wt_base = h.cset.wt_base;
    } else if (h.smoother_precision == 16) {
        h.gset.low_w_base = offbf;
        offbf += h.gset.region;
        h.gset.low_wt_base = offbf;
        offbf += h.gset.region;
        h.cset.low_w_base = offbf;
        offbf += h.cset.region;
        h.cset.low_wt_base = offbf;
        offbf += h.cset.region;
    }
    if (inverse && !lowp) {
        h.gset.s_base = take64(h.gset.region);
        h.cset.s_base = take64(h.cset.region);
        h.gset.low_s_base = h.gset.s_base;
        h.cset.low_s_base = h.cset.s_base;
    }
    h.ar64_n = off64;
    h.ar32_n = off32;
    h.arbf_n = offbf;
    h.grain_region_zero_n = h.gset.region;
    // ---- task lists ---------------------------------------------------------------
    auto Lg = [&](int64_t m, int64_t I, int64_t J) { return h.gset.a_base + h.gset.rel[m] + tri_index(I, J) * TE; };
    auto Rg = [&](int64_t base, int64_t m, int64_t I, int64_t C) { return base + (C * h.gset.nt[m] + I) * TE; };
    auto fg = [&](int64_t m, int64_t I) -> int64_t { return h.gset.first.empty() ? 0 : h.gset.first[(size_t)m][(size_t)I]; };
    // Forward rows of the basis, Y = L^-1 R by substitution (Eq. 23's solves):
    // Y_k = W_kk (R_k - sum_q L_kq Y_q) over the factor's nonzero tiles of row
    // k, in step k of the grain factorisation (after W_kk is formed), R_k
    // entering as the product -I R_k
    std::function<void(int64_t)> y_rows;
    if (h.basis_subst)
        y_rows = [&](int64_t k) {
            for (int64_t m = 0; m < nG; ++m) {
                if (h.gset.nt[m] <= k) continue;
                for (int64_t C = 0; C < h.gm_ntc[(size_t)m]; ++C) {
                    const int32_t ps = (int32_t)h.tl64.pairs.size();
                    for (int64_t q = fg(m, k); q < k; ++q)
                        h.tl64.pairs.push_back({Lg(m, k, q), Rg(h.gm_ytoff[(size_t)m], m, q, C)});
                    h.tl64.pairs.push_back({h.negi_off, Rg(h.gm_roff[(size_t)m], m, k, C)});
                    h.tl64.gemm.push_back({Rg(h.gm_ytoff[(size_t)m], m, k, C),
                                           h.gset.w_base + h.gset.rel[m] + tri_index(k, k) * TE, ps,
                                           (int32_t)(h.tl64.pairs.size() - ps), GF_POST | GF_NEGATE, 0});
                }
            }
        };
    build_factor_program(h.gset, h.tl64, 0, nullptr, nullptr, !h.basis_subst, y_rows);
    if (!c32)
        build_factor_program(h.cset, h.tl64, 1);
    else
        build_factor_program(h.cset, h.tl32, 1);
    TaskLists &tl_inv = !lowp ? h.tl64 : (h.smoother_precision == 32 ? h.tl32 : h.tlbf);
    if (inverse) {
        build_inverse_program(h.gset, tl_inv, lowp);
        build_inverse_program(h.cset, tl_inv, lowp);
    }
    // basis: Y = W R, X = W^T Y (overwrites R), K = Y^T Y, XT = X^T; or by
    // substitution: backward rows X_k = W_kk^T (Y_k - sum_q L_qk^T X_q) over
    // the nonzero tiles L_qk, q > k (X over R, Y_k entering as -I Y_k), one
    // launch per row counted from every matrix's last row, each task also
    // writing X^T, in a program of its own (only the preconditioner's
    // application reads X), and K = Y^T Y, which the coarse operator needs
    {
        std::vector<int64_t> all((size_t)nG);
        std::iota(all.begin(), all.end(), 0);
        if (h.basis_subst) {
            int64_t ntmax = 0;
            for (int64_t m = 0; m < nG; ++m)
                if (h.gm_ntc[(size_t)m] > 0) ntmax = std::max(ntmax, h.gset.nt[m]);
            for (int64_t t = 0; t < ntmax; ++t) {
                Launch L{LK_GEMM, (int64_t)h.tl64.gemm.size(), 0};
                for (int64_t m = 0; m < nG; ++m) {
                    const int64_t nt = h.gset.nt[m], k = nt - 1 - t;
                    if (k < 0) continue;
                    for (int64_t C = 0; C < h.gm_ntc[(size_t)m]; ++C) {
                        const int32_t ps = (int32_t)h.tl64.pairs.size();
                        for (int64_t q = k + 1; q < nt; ++q)
                            if (fg(m, q) <= k) h.tl64.pairs.push_back({Lg(m, q, k), Rg(h.gm_roff[(size_t)m], m, q, C)});
                        h.tl64.pairs.push_back({h.negi_off, Rg(h.gm_ytoff[(size_t)m], m, k, C)});
                        GemmTask task{Rg(h.gm_roff[(size_t)m], m, k, C), h.gset.wt_base + h.gset.wdrel[m] + k * TE,
                                      ps, (int32_t)(h.tl64.pairs.size() - ps), GF_POST | GF_NEGATE | GF_TRANS_A, 0};
                        task.t_off = h.gm_xtoff[(size_t)m] + (k * h.gm_ntc[(size_t)m] + C) * TE;   // X^T
                        h.tl64.gemm.push_back(task);
                    }
                }
                L.count = (int64_t)h.tl64.gemm.size() - L.start;
                if (L.count) h.basis_x_prog.push_back(L);
            }
            append_basis_program(h, h.tl64, all, h.basis_prog, BP_K);
        } else {
            append_basis_program(h, h.tl64, all, h.basis_prog, BP_ALL);
        }
    }
    // apply-time GEMV lists
    {
        if (h.smoother_form == HPLMM_SMOOTHER_INVERSE) {
            build_sym_gemv(h.gset, h.vtasks, h.spairs, h.rtasks, h.sym_part_len, h.gset.low_s_base);
            build_sym_gemv(h.cset, h.vtasks, h.spairs, h.rtasks, h.sym_part_len, h.cset.low_s_base);
        } else {
            const int64_t gw = lowp ? h.gset.low_w_base : h.gset.w_base;
            const int64_t gwt = lowp ? h.gset.low_wt_base : h.gset.wt_base;
            build_smoother_gemv(h.gset, h.vtasks, h.vpairs, gw, gwt);
            const int64_t cw = h.smoother_precision == 16 ? h.cset.low_w_base : h.cset.w_base;
            const int64_t cwt = h.smoother_precision == 16 ? h.cset.low_wt_base : h.cset.wt_base;
            build_smoother_gemv(h.cset, h.vtasks, h.vpairs, cw, cwt);
        }
        // restriction t = X^T x, prolongation z = X u
        h.gemv_XT.start = (int64_t)h.vtasks.size();
        for (int64_t m = 0; m < nG; ++m)
            for (int64_t C = 0; C < h.gm_ntc[(size_t)m]; ++C) {
                h.vtasks.push_back({h.gm_coff[(size_t)m] + C * TS, (int32_t)h.vpairs.size(), (int32_t)h.gset.nt[m], -1});
                for (int64_t I = 0; I < h.gset.nt[m]; ++I)
                    h.vpairs.push_back({h.gm_xtoff[(size_t)m] + (I * h.gm_ntc[(size_t)m] + C) * TE, h.gset.voff[m] + I * TS});
            }
        h.gemv_XT.count = (int64_t)h.vtasks.size() - h.gemv_XT.start;
        h.gemv_X.start = (int64_t)h.vtasks.size();
        for (int64_t m = 0; m < nG; ++m) {
            if (h.gm_ntc[(size_t)m] == 0) continue;
            for (int64_t I = 0; I < h.gset.nt[m]; ++I) {
                h.vtasks.push_back({h.gset.voff[m] + I * TS, (int32_t)h.vpairs.size(), (int32_t)h.gm_ntc[(size_t)m], -1});
                for (int64_t C = 0; C < h.gm_ntc[(size_t)m]; ++C)
                    h.vpairs.push_back({h.gm_roff[(size_t)m] + (C * h.gset.nt[m] + I) * TE, h.gm_coff[(size_t)m] + C * TS});
            }
        }
        h.gemv_X.count = (int64_t)h.vtasks.size() - h.gemv_X.start;
    }
    split_program(h.gset.factor_prog, h.tl64);
    split_program(h.gset.w_prog, h.tl64);
    split_program(h.cset.factor_prog, c32 ? h.tl32 : h.tl64);
    split_program(h.basis_prog, h.tl64);
    split_program(h.basis_x_prog, h.tl64);
    split_program(h.gset.inverse_prog, tl_inv);
    split_program(h.cset.inverse_prog, tl_inv);
    fill_flops(h.gset.inverse_prog, tl_inv);
    fill_flops(h.cset.inverse_prog, tl_inv);
    fill_flops(h.gset.factor_prog, h.tl64);
    fill_flops(h.gset.w_prog, h.tl64);
    fill_flops(h.cset.factor_prog, c32 ? h.tl32 : h.tl64);
    fill_flops(h.basis_prog, h.tl64);
    fill_flops(h.basis_x_prog, h.tl64);
    {
        const double ge = h.smoother_precision == 64 ? 8.0 : (h.smoother_precision == 32 ? 4.0 : 2.0);
        // S of the reduced-precision inverse form is kept in FP32
        const double gs = h.smoother_precision == 64 ? 8.0 : 4.0;
        h.gset.gemv_W.bytes = gemv_bytes(h.vtasks, h.gset.gemv_W, ge);
        h.gset.gemv_Wt.bytes = gemv_bytes(h.vtasks, h.gset.gemv_Wt, ge);
        h.cset.gemv_W.bytes = gemv_bytes(h.vtasks, h.cset.gemv_W, ge);
        h.cset.gemv_Wt.bytes = gemv_bytes(h.vtasks, h.cset.gemv_Wt, ge);
        for (DenseSet *ds : {&h.gset, &h.cset}) {
            ds->gemv_S.bytes = sym_gemv_bytes(h.vtasks, h.spairs, ds->gemv_S, gs);
            ds->red_S.bytes = sym_reduce_bytes(h.rtasks, ds->red_S);
        }
        h.gemv_XT.bytes = gemv_bytes(h.vtasks, h.gemv_XT, 8.0);
        h.gemv_X.bytes = gemv_bytes(h.vtasks, h.gemv_X, 8.0);
        // fine SpMV: 72 B of values + 4 B of index per stored block, x read and
        // y written once, row pointer
        h.spmv_bytes = (double)h.nnzb * 76.0 + (double)n * (24.0 + 24.0 + 8.0);
        // one application of M^-1 (Eq. 16): the operators above once each, two
        // residual SpMVs (which also read r), and the vector gathers/combines
        h.apply_bytes = h.gset.gemv_W.bytes + h.gset.gemv_Wt.bytes + h.cset.gemv_W.bytes +
                        h.cset.gemv_Wt.bytes + h.gset.gemv_S.bytes + h.cset.gemv_S.bytes +
                        h.gemv_XT.bytes + h.gemv_X.bytes + 2.0 * (h.spmv_bytes + 24.0 * n) +
                        8.0 * (6.0 * h.N + 3.0 * (double)h.gset.vec_len + 2.0 * (double)h.cset.vec_len);
    }
    pad_ones(h.gset, h.pad_ones_g, h.gset.a_base);
    pad_ones(h.cset, h.pad_ones_c, c32 ? h.c_stage_base : h.cset.a_base);
    // ---- index maps ------------------------------------------------------------------
    const int64_t s_pad = h.n_mortar;   // corrections follow the mortar dofs
    h.cvec_len = s_pad + h.n_corr;
    std::vector<int64_t> fpos((size_t)h.n_coarse);
    for (int64_t q = 0; q < h.n_mortar; ++q) fpos[(size_t)q] = q;
    for (int64_t j = 0; j < h.n_corr; ++j) fpos[(size_t)(h.n_mortar + j)] = s_pad + j;
    std::vector<int32_t> q_iface((size_t)h.n_mortar), q_local((size_t)h.n_mortar);
    for (int32_t c = 0; c < part.n_ifaces; ++c)
        for (int32_t j = 0; j < 3 * iface_nu[(size_t)c]; ++j) {
            q_iface[(size_t)(iface_moff[(size_t)c] + j)] = c;
            q_local[(size_t)(iface_moff[(size_t)c] + j)] = j;
        }
    // t-slot lists: grains adjacent to the interface of each mortar dof, ascending
    std::vector<std::vector<int32_t>> iface_gm((size_t)part.n_ifaces);
    for (int64_t m = 0; m < nG; ++m)
        for (int32_t c : gadj[(size_t)m]) iface_gm[(size_t)c].push_back((int32_t)m);
    std::vector<int64_t> tptr(1, 0), tslot;
    for (int64_t q = 0; q < h.n_mortar; ++q) {
        const int32_t c = q_iface[(size_t)q];
        for (int32_t m : iface_gm[(size_t)c]) tslot.push_back(h.gm_coff[(size_t)m] + lcol[(size_t)m][c] + q_local[(size_t)q]);
        tptr.push_back((int64_t)tslot.size());
    }
    std::vector<int64_t> corr_koff;
    for (int64_t m = 0; m < nG; ++m) {
        const int32_t j = h.gm_corr[(size_t)m];
        if (j < 0) continue;
        (void)j;
    }
    for (int64_t j = 0; j < h.n_corr; ++j) {
        const int32_t m = grain_mat[(size_t)h.h_corr_grains[(size_t)j]];
        const int64_t kc = h.gm_k[(size_t)m];
        tslot.push_back(h.gm_coff[(size_t)m] + kc);
        tptr.push_back((int64_t)tslot.size());
        corr_koff.push_back(h.gm_koff[(size_t)m] + tri_index(kc / TS, kc / TS) * TE + (kc % TS) * TS + (kc % TS));
    }
    std::vector<int64_t> gcol_upos((size_t)std::max<int64_t>(h.gcol_len, 1), -1);
    for (int64_t m = 0; m < nG; ++m) {
        for (int32_t c : gadj[(size_t)m])
            for (int32_t j = 0; j < 3 * iface_nu[(size_t)c]; ++j)
                gcol_upos[(size_t)(h.gm_coff[(size_t)m] + lcol[(size_t)m][c] + j)] = iface_moff[(size_t)c] + j;
        if (h.gm_corr[(size_t)m] >= 0)
            gcol_upos[(size_t)(h.gm_coff[(size_t)m] + h.gm_k[(size_t)m])] = s_pad + h.gm_corr[(size_t)m];
    }
    std::vector<int64_t> g_slot_dof((size_t)std::max<int64_t>(h.gset.vec_len, 1), -1), g_dof_slot((size_t)h.N, -1);
    for (int64_t m = 0; m < nG; ++m) {
        auto &nodes = gnodes[(size_t)h.gm_grain[(size_t)m]];
        for (size_t l = 0; l < nodes.size(); ++l)
            for (int d = 0; d < 3; ++d) {
                const int64_t slot = h.gset.voff[m] + 3 * (int64_t)l + d, dof = 3 * (int64_t)nodes[l] + d;
                g_slot_dof[(size_t)slot] = dof;
                g_dof_slot[(size_t)dof] = slot;
            }
    }
    // contacts: per-node membership (ascending contact id) and slot maps
    for (int64_t v = 0; v < n; ++v) cn_cnt[(size_t)v + 1] += cn_cnt[(size_t)v];
    std::vector<int32_t> node_cmat((size_t)std::max<int64_t>(cn_cnt[(size_t)n], 1)), node_cloc(node_cmat.size());
    std::vector<int32_t> item_node, item_mat, item_local;
    {
        std::vector<int64_t> fill(cn_cnt.begin(), cn_cnt.end() - 1);
        for (int32_t c = 0; c < part.n_contacts; ++c)
            for (int64_t p = part.contact_ptr[c]; p < part.contact_ptr[c + 1]; ++p) {
                const int32_t v = part.contact_nodes[p];
                const int32_t l = (int32_t)(p - part.contact_ptr[c]);
                node_cmat[(size_t)fill[(size_t)v]] = c;
                node_cloc[(size_t)fill[(size_t)v]++] = l;
                item_node.push_back(v);
                item_mat.push_back(c);
                item_local.push_back(l);
            }
    }
    std::vector<int64_t> c_slot_dof((size_t)std::max<int64_t>(h.cset.vec_len, 1), -1);
    std::vector<int64_t> c_dof_ptr((size_t)h.N + 1, 0), c_dof_slot;
    for (int32_t c = 0; c < part.n_contacts; ++c)
        for (int64_t p = part.contact_ptr[c]; p < part.contact_ptr[c + 1]; ++p)
            for (int d = 0; d < 3; ++d)
                c_slot_dof[(size_t)(h.cset.voff[c] + 3 * (p - part.contact_ptr[c]) + d)] = 3 * (int64_t)part.contact_nodes[p] + d;
    for (int64_t v = 0; v < n; ++v)
        for (int d = 0; d < 3; ++d) {
            for (int64_t q = cn_cnt[(size_t)v]; q < cn_cnt[(size_t)v + 1]; ++q)
                c_dof_slot.push_back(h.cset.voff[node_cmat[(size_t)q]] + 3 * (int64_t)node_cloc[(size_t)q] + d);
            c_dof_ptr[(size_t)(3 * v + d + 1)] = (int64_t)c_dof_slot.size();
        }
    // coarse Galerkin pairs: interface-interface edges of A and shared grains
    std::vector<CoarseEdge> edges;
    std::vector<CoarseKRef> krefs;
    std::vector<CoarsePair> pairs;
    {
        struct EdgeKey {
            int64_t key;
            CoarseEdge e;
        };
        std::vector<EdgeKey> ek;
        const int64_t NI = std::max<int32_t>(part.n_ifaces, 1);
        for (int64_t v = 0; v < n; ++v) {
            const int32_t c = node_iface[(size_t)v];
            if (c < 0) continue;
            for (int64_t p = sys.row_ptr[v]; p < sys.row_ptr[v + 1]; ++p) {
                const int32_t w = sys.col_idx[p];
                const int32_t c2 = node_iface[(size_t)w];
                if (c2 < 0 || c2 > c) continue;
                ek.push_back({(int64_t)c * NI + c2, {p, node_irow[(size_t)v], node_irow[(size_t)w]}});
            }
        }
        std::stable_sort(ek.begin(), ek.end(), [](const EdgeKey &a, const EdgeKey &b) { return a.key < b.key; });
        struct KKey {
            int64_t key;
            CoarseKRef r;
        };
        std::vector<KKey> kk;
        for (int64_t m = 0; m < nG; ++m) {
            auto &a = gadj[(size_t)m];
            for (size_t i = 0; i < a.size(); ++i)
                for (size_t j = 0; j <= i; ++j)
                    kk.push_back({(int64_t)a[i] * NI + a[j],
                                  {h.gm_koff[(size_t)m], lcol[(size_t)m][a[i]], lcol[(size_t)m][a[j]]}});
        }
        std::stable_sort(kk.begin(), kk.end(), [](const KKey &a, const KKey &b) { return a.key < b.key; });
        size_t ie = 0, ik = 0;
        while (ie < ek.size() || ik < kk.size()) {
            int64_t key = INT64_MAX;
            if (ie < ek.size()) key = std::min(key, ek[ie].key);
            if (ik < kk.size()) key = std::min(key, kk[ik].key);
            CoarsePair pr{};
            pr.c = (int32_t)(key / NI);
            pr.c2 = (int32_t)(key % NI);
            pr.e_start = (int64_t)edges.size();
            while (ie < ek.size() && ek[ie].key == key) edges.push_back(ek[ie++].e);
            pr.e_count = (int32_t)((int64_t)edges.size() - pr.e_start);
            pr.k_start = (int64_t)krefs.size();
            while (ik < kk.size() && kk[ik].key == key) krefs.push_back(kk[ik++].r);
            pr.k_count = (int32_t)((int64_t)krefs.size() - pr.k_start);
            pairs.push_back(pr);
        }
    }
    // ---- multifrontal coarse factorisation plan ---------------------------------------
    build_coarse_mf(h, sys, part, iface_nu, iface_moff, pairs, off64);
    h.ar64_n = off64;
    h.h_pairs = pairs;
    {
        // one application also runs the coarse forward and backward sweeps over
        // the front factors (W11 and G, then W11^T and G^T) and their vectors
        h.apply_bytes += 2.0 * h.mf.factor_bytes + 8.0 * 8.0 * (double)h.mf.vec_len;
    }
    method_work(h);
    // ---- SELL-64 fine matrix ---------------------------------------------------------
    std::vector<int64_t> slice_step;
    std::vector<int32_t> scol;
    std::vector<double> sval;
    {
        const int64_t ns = (n + SELL_C - 1) / SELL_C;
        slice_step.resize((size_t)ns + 1, 0);
        for (int64_t sl = 0; sl < ns; ++sl) {
            int64_t len = 0;
            for (int64_t r = sl * SELL_C; r < std::min(n, (sl + 1) * SELL_C); ++r)
                len = std::max(len, sys.row_ptr[r + 1] - sys.row_ptr[r]);
            slice_step[(size_t)sl + 1] = slice_step[(size_t)sl] + len;
        }
        const int64_t steps = slice_step[(size_t)ns];
        scol.assign((size_t)steps * SELL_C, 0);
        sval.assign((size_t)steps * 9 * SELL_C, 0.0);
        for (int64_t sl = 0; sl < ns; ++sl)
            for (int64_t lane = 0; lane < SELL_C; ++lane) {
                const int64_t r = sl * SELL_C + lane;
                for (int64_t k = slice_step[(size_t)sl]; k < slice_step[(size_t)sl + 1]; ++k) {
                    const int64_t kk = k - slice_step[(size_t)sl];
                    int64_t col = r < n ? r : 0;
                    const double *blk = nullptr;
                    if (r < n && kk < sys.row_ptr[r + 1] - sys.row_ptr[r]) {
                        col = sys.col_idx[sys.row_ptr[r] + kk];
                        blk = sys.val + 9 * (sys.row_ptr[r] + kk);
                    }
                    scol[(size_t)(k * SELL_C + lane)] = (int32_t)col;
                    for (int j = 0; j < 9; ++j)
                        sval[(size_t)(k * 9 * SELL_C + j * SELL_C + lane)] = blk ? blk[j] : 0.0;
                }
            }
        h.sell_padded_blocks = steps * SELL_C;
        h.sell.n_rows = n;
        h.sell.n_slices = (int32_t)ns;
    }

    // ---- bounds validation of every launch list and index map ------------------------
    {
        auto chk = [](bool ok, const char *what) {
            if (!ok) fail(HPLMM_E_ARG, std::string("internal plan check failed: ") + what);
        };
        auto in = [](int64_t off, int64_t len, int64_t n) { return off >= 0 && off + len <= n; };
        for (int which = 0; which < 3; ++which) {
            // the bfloat16 list reads the bfloat16 arena and writes the FP32 one
            const TaskLists &tl = which == 2 ? h.tlbf : which ? h.tl32 : h.tl64;
            const int64_t an = which == 2 ? h.arbf_n : which ? h.ar32_n : h.ar64_n;
            const int64_t on = which ? h.ar32_n : h.ar64_n;
            for (const auto &t : tl.gemm) {
                chk(in(t.c_off, TE, on), "gemm output tile");
                if (t.t_off >= 0)
                    chk(in(t.t_off, TE, on) && (!(t.flags & GF_ACCUM) || (t.flags & (GF_POST | GF_POST_RIGHT))),
                        "gemm transposed output tile");
                else
                    chk(t.t_off == -1, "gemm transposed output tile");
                if (which == 2) chk(!(t.flags & (GF_POST | GF_POST_RIGHT)), "bfloat16 task without second product");
                if (t.flags & (GF_POST | GF_POST_RIGHT)) chk(in(t.post_off, TE, an), "gemm post tile");
                chk(t.pair_start >= 0 && t.pair_count >= 0 && (int64_t)t.pair_start + t.pair_count <= (int64_t)tl.pairs.size(),
                    "gemm pair range");
                if (t.nchunk > 1)
                    chk(t.chunk >= 0 && t.chunk < t.nchunk && t.part_off >= 0 &&
                            t.part_off + (int64_t)t.nchunk * TE <= tl.part_len,
                        "gemm split task");
                else
                    chk(t.nchunk == 1 && t.chunk == 0, "gemm task");
            }
            for (const auto &pr : tl.pairs) chk(in(pr.a_off, TE, an) && in(pr.b_off, TE, an), "gemm operand tile");
            for (const auto &d : tl.diag)
                chk(in(d.a_off, TE, an) && in(d.w_off, TE, an) && in(d.wt_off, TE, an) && (d.p_off < 0 || in(d.p_off, TE, an)),
                    "diag tile");
            for (const auto &c : tl.copy) chk(in(c.src_off, TE, an) && in(c.dst_off, TE, an), "transpose tile");
        }
        const int64_t low_n = h.smoother_precision == 32 ? h.ar32_n : (h.smoother_precision == 16 ? h.arbf_n : h.ar64_n);
        const int64_t c_n = h.smoother_precision == 64 ? h.ar64_n : (h.smoother_precision == 32 ? h.ar32_n : h.arbf_n);
        auto chk_gemv = [&](Range r, int64_t an, int64_t xl, int64_t yl, const char *what) {
            bool any_split = false;
            for (int64_t i = r.start; i < r.start + r.count; ++i) {
                const GemvTask &t = h.vtasks[(size_t)i];
                chk(in(t.y_off, TS, yl), what);
                chk(t.base_off < 0 || in(t.base_off, TS, yl), what);
                if (t.nchunk > 1) {
                    any_split = true;
                    chk(t.chunk >= 0 && t.chunk < t.nchunk && t.part_off >= 0 &&
                            t.part_off + (int64_t)t.nchunk * TS <= h.gemv_part_len,
                        what);
                    // the reduction launch reads a row's partials from its first
                    // chunk: the row's chunks follow it, in order, in this launch
                    if (t.chunk == 0) {
                        chk(i + t.nchunk <= r.start + r.count, what);
                        for (int64_t c = 1; c < t.nchunk && i + c < r.start + r.count; ++c) {
                            const GemvTask &u = h.vtasks[(size_t)(i + c)];
                            chk(u.chunk == c && u.nchunk == t.nchunk && u.y_off == t.y_off &&
                                    u.base_off == t.base_off && u.part_off == t.part_off,
                                what);
                        }
                    }
                } else {
                    chk(t.nchunk == 1 && t.chunk == 0, what);
                }
                chk(t.pair_start >= 0 && (int64_t)t.pair_start + t.pair_count <= (int64_t)h.vpairs.size(), what);
                for (int32_t q = 0; q < t.pair_count; ++q) {
                    const GemvPair &pr = h.vpairs[(size_t)(t.pair_start + q)];
                    chk(in(pr.t_off, TE, an) && in(pr.x_off, TS, xl), what);
                }
            }
            // the reduction launch follows exactly the launches with split rows
            chk(any_split == r.split, what);
        };
        chk_gemv(h.gset.gemv_W, low_n, h.gset.vec_len, h.gset.vec_len, "grain W gemv");
        chk_gemv(h.gset.gemv_Wt, low_n, h.gset.vec_len, h.gset.vec_len, "grain Wt gemv");
        chk_gemv(h.cset.gemv_W, c_n, h.cset.vec_len, h.cset.vec_len, "contact W gemv");
        chk_gemv(h.cset.gemv_Wt, c_n, h.cset.vec_len, h.cset.vec_len, "contact Wt gemv");
        auto chk_sym = [&](const DenseSet &ds, const char *what) {
            const Range r = ds.gemv_S;
            for (int64_t i = r.start; i < r.start + r.count; ++i) {
                const GemvTask &t = h.vtasks[(size_t)i];
                chk(in(t.y_off, TS, ds.vec_len) && t.base_off < 0 && t.nchunk == 1 && t.chunk == 0, what);
                chk(t.pair_start >= 0 && t.pair_count >= 1 && (int64_t)t.pair_start + t.pair_count <= (int64_t)h.spairs.size(),
                    what);
                for (int32_t q = 0; q < t.pair_count; ++q) {
                    const SymPair &pr = h.spairs[(size_t)(t.pair_start + q)];
                    chk(in(pr.t_off, TE, h.smoother_precision == 64 ? h.ar64_n : h.ar32_n) &&
                            in(pr.x_off, TS, ds.vec_len) && pr.rows >= 1 && pr.rows <= TS && pr.cols >= 1 &&
                            pr.cols <= TS,
                        what);
                    // the diagonal tile, last in its row, carries no transposed product
                    chk(q + 1 == t.pair_count ? pr.p_off == -1 : in(pr.p_off, TS, h.sym_part_len), what);
                }
            }
            for (int64_t i = ds.red_S.start; i < ds.red_S.start + ds.red_S.count; ++i) {
                const SymReduce &t = h.rtasks[(size_t)i];
                chk(t.count >= 1 && in(t.y_off, TS, ds.vec_len) && in(t.p_off, (int64_t)t.count * TS, h.sym_part_len), what);
            }
        };
        if (h.smoother_form == HPLMM_SMOOTHER_INVERSE) {
            // S in the FP64 arena at full precision, in the FP32 one otherwise
            chk(h.smoother_precision == 64 ? h.gset.s_base >= 0 && h.cset.s_base >= 0
                                           : h.gset.s_base < 0 && h.cset.s_base < 0,
                "inverse regions");
            chk_sym(h.gset, "grain S gemv");
            chk_sym(h.cset, "contact S gemv");
        } else {
            chk(h.gset.gemv_S.count == 0 && h.cset.gemv_S.count == 0, "symmetric lists in the factor form");
        }
        chk_gemv(h.gemv_XT, h.ar64_n, h.gset.vec_len, h.gcol_len, "restriction gemv");
        chk_gemv(h.gemv_X, h.ar64_n, h.gcol_len, h.gset.vec_len, "prolongation gemv");
        for (auto v : g_slot_dof) chk(v >= -1 && v < h.N, "grain slot map");
        for (auto v : g_dof_slot) chk(v >= -1 && v < h.gset.vec_len, "grain dof map");
        for (auto v : gcol_upos) chk(v >= -1 && v < h.cvec_len, "grain column map");
        for (auto v : c_slot_dof) chk(v >= -1 && v < h.N, "contact slot map");
        for (auto v : c_dof_slot) chk(v >= 0 && v < h.cset.vec_len, "contact dof map");
        for (auto v : fpos) chk(v >= 0 && v < h.cvec_len, "coarse position map");
        for (auto v : tslot) chk(v >= 0 && v < h.gcol_len, "restriction slot map");
        for (auto v : corr_koff) chk(in(v, 1, h.ar64_n), "correction pivot offset");
        for (auto v : h.pad_ones_g) chk(in(v, 1, h.ar64_n), "grain padding");
        for (auto v : h.pad_ones_c) chk(in(v, 1, h.ar64_n), "contact padding");
        for (auto v : scol) chk(v >= 0 && v < n, "SELL column");
        for (const auto &e : edges) chk(e.blk >= 0 && e.blk < h.nnzb, "coarse edge block");
        for (const auto &k : krefs) chk(in(k.koff, 1, h.ar64_n), "coarse K reference");
        for (const auto &w : abar) chk(w.m >= 0 && w.m < nG && w.lcol0 >= 0 && w.lcol0 < h.gm_k[(size_t)w.m], "abar work");
        for (int64_t m = 0; m < nG; ++m) {
            chk(in(h.gm_roff[(size_t)m], h.gset.nt[m] * h.gm_ntc[(size_t)m] * TE, h.ar64_n), "R region");
            chk(in(h.gm_koff[(size_t)m], tri_tiles(h.gm_ntc[(size_t)m]) * TE, h.ar64_n), "K region");
        }
        chk(in(h.gset.a_base, h.gset.region, h.ar64_n), "grain region");
        chk(h.n_coarse <= h.cvec_len, "coarse vector length");
        {
            const CoarseMF &mf = h.mf;
            for (const auto &r : mf.ext) {
                chk(in(r.parent_off, TE, h.ar64_n) && r.PI >= r.PJ && r.PJ >= 0 && r.PI < r.ntp, "extend-add tile");
                for (int s = 0; s < 2; ++s)
                    if (r.child_off[s] >= 0)
                        chk(in(r.inv_off[s], (int64_t)r.ntp * TS, (int64_t)mf.inv.size()) && r.nt_d[s] >= 0,
                            "extend-add child");
                    else
                        chk(r.child_off[s] == -1, "extend-add child");
            }
            for (int32_t t = 0; t < mf.n_fronts; ++t) {
                const int64_t nt = mf.nt_d[(size_t)t] + mf.nt_u[(size_t)t];
                chk(in(mf.a_base + mf.rel[(size_t)t], tri_tiles(nt) * TE, h.ar64_n), "front tiles");
                chk(in(mf.wrel[(size_t)t], tri_tiles(mf.nt_d[(size_t)t]) * TE, mf.w_region) &&
                        mf.wt_base == mf.w_base + mf.w_region && in(mf.wt_base, mf.w_region, h.ar64_n),
                    "front W11 tiles");
                chk(in(mf.lt_base + mf.ltrel[(size_t)t], mf.nt_d[(size_t)t] * mf.nt_u[(size_t)t] * TE, h.ar64_n),
                    "front NG^T tiles");
                chk(in(mf.ng_base + mf.ltrel[(size_t)t], mf.nt_d[(size_t)t] * mf.nt_u[(size_t)t] * TE, h.ar64_n),
                    "front NG tiles");
            }
            // every extend-add position lies inside the parent front
            std::unordered_map<int64_t, int64_t> front_nt;
            for (int32_t t = 0; t < mf.n_fronts; ++t)
                front_nt[mf.a_base + mf.rel[(size_t)t]] = mf.nt_d[(size_t)t] + mf.nt_u[(size_t)t];
            const std::vector<int64_t> &inv_at = mf.inv_at;
            chk((int64_t)inv_at.size() == (int64_t)mf.n_fronts, "extend-add inverse maps");
            std::unordered_map<int64_t, int32_t> front_of;
            for (int32_t t = 0; t < mf.n_fronts; ++t) front_of[mf.a_base + mf.rel[(size_t)t]] = t;
            for (const auto &r : mf.ext) {
                auto it = front_nt.find(r.parent_off - tri_index(r.PI, r.PJ) * TE);
                chk(it != front_nt.end() && it->second == r.ntp, "extend-add parent front");
                for (int s = 0; s < 2; ++s) {
                    if (r.child_off[s] < 0) continue;
                    auto ic = front_of.find(r.child_off[s]);
                    chk(ic != front_of.end(), "extend-add child front");
                    const int32_t ch = ic->second;
                    chk(r.nt_d[s] == mf.nt_d[(size_t)ch] && mf.parent[(size_t)ch] >= 0 &&
                            mf.a_base + mf.rel[(size_t)mf.parent[(size_t)ch]] == it->first && r.inv_off[s] == inv_at[(size_t)ch],
                        "extend-add child");
                }
            }
            // every child row an inverse map names lies in the child's boundary block
            for (int32_t t = 0; t < mf.n_fronts; ++t) {
                const int32_t par = mf.parent[(size_t)t];
                if (par < 0) continue;
                chk(mf.u[(size_t)t] <= mf.nt_u[(size_t)t] * TS, "extend-add child rows");
                const int64_t np = (mf.nt_d[(size_t)par] + mf.nt_u[(size_t)par]) * TS;
                chk(in(inv_at[(size_t)t], np, (int64_t)mf.inv.size()), "extend-add inverse map");
                for (int64_t p = 0; p < np; ++p) {
                    const int32_t v = mf.inv[(size_t)(inv_at[(size_t)t] + p)];
                    chk(v >= -1 && v < mf.u[(size_t)t], "extend-add child row");
                }
            }
            for (auto v : mf.maps) chk(v >= 0, "extend-add position");
            for (auto v : mf.va_dst) chk(in(v, 1, mf.vec_len), "front vector extend-add");
            for (auto v : mf.va_src) chk(in(v, 1, mf.vec_len), "front vector extend-add source");
            for (auto v : mf.cp_dst) chk(in(v, 1, mf.vec_len), "front vector copy");
            for (auto v : mf.cp_src) chk(in(v, 1, mf.vec_len), "front vector copy source");
            for (auto v : mf.init_map) chk(v >= -1 && v < h.cvec_len, "front right-hand side map");
            for (auto v : mf.out_dst) chk(in(v, 1, h.cvec_len), "coarse solution map");
            for (auto v : mf.out_src) chk(in(v, 1, mf.vec_len), "coarse solution source");
            for (auto v : mf.pad_ones) chk(in(v, 1, h.ar64_n), "front padding");
            for (int32_t l = 0; l < mf.n_levels; ++l) {
                chk_gemv(mf.fwd[(size_t)l], h.ar64_n, 3 * mf.vec_len, 3 * mf.vec_len, "front forward sweep");
                chk_gemv(mf.bwd[(size_t)l], h.ar64_n, 3 * mf.vec_len, 3 * mf.vec_len, "front backward sweep");
                // every launch shape the autotuner may pick
                for (const Range &v : mf.fwd_shapes[(size_t)l].var)
                    chk_gemv(v, h.ar64_n, 3 * mf.vec_len, 3 * mf.vec_len, "front forward sweep shape");
                for (const Range &v : mf.bwd_shapes[(size_t)l].var)
                    chk_gemv(v, h.ar64_n, 3 * mf.vec_len, 3 * mf.vec_len, "front backward sweep shape");
            }
            for (const auto &pr : pairs) {
                chk(in(pr.f_off, 1, h.ar64_n), "coarse pair front");
                chk(pr.v_off >= 0 && pr.v_off + 9 * (int64_t)iface_nu[(size_t)pr.c] * iface_nu[(size_t)pr.c2] <= h.n_pair_vals,
                    "coarse pair values");
            }
        }
    }
    if (dry_run) return;
    // ---- uploads --------------------------------------------------------------------------
    std::vector<int64_t> rp(sys.row_ptr, sys.row_ptr + n + 1);
    std::vector<int32_t> ci(sys.col_idx, sys.col_idx + h.nnzb);
    std::vector<double> va(sys.val, sys.val + 9 * h.nnzb);
    h.csr.n_nodes = n;
    h.csr.row_ptr = h.upload(rp, s);
    h.csr.col = h.upload(ci, s);
    h.csr.val = h.upload(va, s);
    h.sell.slice_step = h.upload(slice_step, s);
    h.sell.col = h.upload(scol, s);
    h.sell.val = h.upload(sval, s);
    std::vector<double> bvec((size_t)h.N, 0.0);
    if (sys.rhs) std::memcpy(bvec.data(), sys.rhs, sizeof(double) * (size_t)h.N);
    h.d_b = h.upload(bvec, s);
    // coarse maps
    h.cm.n_ifaces = h.n_ifaces;
    h.cm.n_mortar = h.n_mortar;
    h.cm.n_coarse = h.n_coarse;
    h.cm.fpos = h.upload(fpos, s);
    h.cm.q_iface = h.upload(q_iface, s);
    h.cm.q_local = h.upload(q_local, s);
    std::vector<int64_t> ip(part.iface_ptr, part.iface_ptr + part.n_ifaces + 1);
    std::vector<int32_t> inodes(part.iface_nodes, part.iface_nodes + (part.n_ifaces ? part.iface_ptr[part.n_ifaces] : 0));
    h.cm.iface_ptr = h.upload(ip, s);
    h.cm.iface_nodes = h.upload(inodes, s);
    h.cm.iface_hoff = h.upload(iface_hoff, s);
    h.cm.iface_nu = h.upload(iface_nu, s);
    h.cm.iface_moff = h.upload(iface_moff, s);
    h.cm.H = h.upload(h.h_H, s);
    h.cm.general = h.mortar_kind == HPLMM_MORTAR_ALGEBRAIC ? 1 : 0;
    h.cm.tptr = h.upload(tptr, s);
    h.cm.tslot = h.upload(tslot, s);
    h.corr_d = h.dalloc<double>(h.n_corr);
    h.cm.corr_d = h.corr_d;
    h.cm.node_iface = h.upload(node_iface, s);
    h.cm.node_irow = h.upload(node_irow, s);
    h.d_corr_koff = h.upload(corr_koff, s);
    // grains
    h.gg.node_gmat = h.upload(node_gmat, s);
    h.gg.node_local = h.upload(node_local, s);
    std::vector<int64_t> aoff(nG);
    std::vector<int32_t> nt32(nG), corrcol(nG);
    for (int64_t m = 0; m < nG; ++m) {
        aoff[(size_t)m] = h.gset.a_base + h.gset.rel[m];
        nt32[(size_t)m] = (int32_t)h.gset.nt[m];
        corrcol[(size_t)m] = h.gm_corr[(size_t)m] >= 0 ? h.gm_k[(size_t)m] : -1;
    }
    h.gg.mat_aoff = h.upload(aoff, s);
    h.gg.mat_roff = h.upload(h.gm_roff, s);
    h.gg.mat_nt = h.upload(nt32, s);
    h.gg.mat_corrcol = h.upload(corrcol, s);
    h.n_abar = (int64_t)abar.size();
    h.d_abar = h.upload(abar, s);
    h.d_g_slot_dof = h.upload(g_slot_dof, s);
    h.d_g_dof_slot = h.upload(g_dof_slot, s);
    h.d_gcol_upos = h.upload(gcol_upos, s);
    h.d_pad_g = h.upload(h.pad_ones_g, s);
    // the tiles a gather and the factorisation can touch: row I of matrix m
    // from its envelope's first column to the diagonal, contiguous in the
    // packed lower-tile layout; runs of at most ZERO_RUN elements
    auto envelope_runs = [](const DenseSet &ds, int64_t base, std::vector<int64_t> &runs) {
        runs.clear();
        if (ds.first.empty() || (base & 1)) return;
        int64_t o0 = -1, o1 = -1;
        auto flush = [&] {
            for (int64_t o = o0; o < o1; o += ZERO_RUN) {
                runs.push_back(o);
                runs.push_back(std::min(ZERO_RUN, o1 - o));
            }
        };
        for (size_t m = 0; m < ds.n.size(); ++m)
            for (int64_t I = 0; I < ds.nt[m]; ++I) {
                const int64_t J0 = ds.first[m][(size_t)I];
                const int64_t a = base + ds.rel[m] + tri_index(I, J0) * TE, b = base + ds.rel[m] + tri_index(I, I + 1) * TE;
                if (a == o1) {
                    o1 = b;
                } else {
                    if (o0 >= 0) flush();
                    o0 = a;
                    o1 = b;
                }
            }
        if (o0 >= 0) flush();
        for (size_t i = 0; i < runs.size(); i += 2)
            if (runs[i] < base || runs[i + 1] <= 0 || runs[i + 1] > ZERO_RUN || (runs[i] & 1) || (runs[i + 1] & 1) ||
                runs[i] + runs[i + 1] > base + ds.region)
                fail(HPLMM_E_ARG, "internal plan check failed: envelope zero run");
    };
    envelope_runs(h.gset, h.gset.a_base, h.zero_g);
    h.d_zero_g = h.upload(h.zero_g, s);
    if (!c32) {
        envelope_runs(h.cset, h.cset.a_base, h.zero_c);
        h.d_zero_c = h.upload(h.zero_c, s);
    }
    // contacts
    std::vector<int64_t> caoff(h.cset.n.size());
    for (size_t m = 0; m < h.cset.n.size(); ++m) caoff[m] = (c32 ? h.c_stage_base : h.cset.a_base) + h.cset.rel[m];
    h.cg.mat_aoff = h.upload(caoff, s);
    h.cg.item_node = h.upload(item_node, s);
    h.cg.item_mat = h.upload(item_mat, s);
    h.cg.item_local = h.upload(item_local, s);
    h.cg.node_cptr = h.upload(cn_cnt, s);
    h.cg.node_cmat = h.upload(node_cmat, s);
    h.cg.node_cloc = h.upload(node_cloc, s);
    h.n_citems = (int64_t)item_node.size();
    h.d_c_slot_dof = h.upload(c_slot_dof, s);
    h.d_c_dof_ptr = h.upload(c_dof_ptr, s);
    h.d_c_dof_slot = h.upload(c_dof_slot, s);
    h.d_pad_c = h.upload(h.pad_ones_c, s);
    // coarse
    h.n_pairs = (int64_t)pairs.size();
    h.d_pairs = h.upload(pairs, s);
    h.d_edges = h.upload(edges, s);
    h.d_krefs = h.upload(krefs, s);
    h.pair_vals = h.dalloc<double>(h.n_pair_vals);
    {
        CoarseMF &mf = h.mf;
        mf.d_ext = h.upload(mf.ext, s);
        mf.d_inv = h.upload(mf.inv, s);
        mf.d_va_dst = h.upload(mf.va_dst, s);
        mf.d_va_ptr = h.upload(mf.va_ptr, s);
        mf.d_va_src = h.upload(mf.va_src, s);
        mf.d_cp_dst = h.upload(mf.cp_dst, s);
        mf.d_cp_src = h.upload(mf.cp_src, s);
        mf.d_init_map = h.upload(mf.init_map, s);
        mf.d_out_dst = h.upload(mf.out_dst, s);
        mf.d_out_src = h.upload(mf.out_src, s);
        mf.d_pad = h.upload(mf.pad_ones, s);
        mf.V = h.dalloc<double>(3 * mf.vec_len);
        mf.WV = mf.V;
        mf.YV = mf.V + mf.vec_len;
        mf.XV = mf.V + 2 * mf.vec_len;
        // padding slots of the front vectors are never written and must read as 0
        if (mf.vec_len > 0 && hipMemsetAsync(mf.V, 0, sizeof(double) * 3 * (size_t)mf.vec_len, s) != hipSuccess)
            fail(HPLMM_E_HIP, "hipMemsetAsync failed");
    }
    // task lists
    for (TaskLists *tl : {&h.tl64, &h.tl32, &h.tlbf}) {
        tl->d_gemm = h.upload(tl->gemm, s);
        tl->d_pairs = h.upload(tl->pairs, s);
        tl->d_diag = h.upload(tl->diag, s);
        tl->d_copy = h.upload(tl->copy, s);
    }
    h.tl64.d_part = h.dalloc<double>(std::max<int64_t>(1, h.tl64.part_len));
    h.tl32.d_part = h.dalloc<float>(std::max<int64_t>(1, h.tl32.part_len));
    h.tlbf.d_part = h.dalloc<float>(std::max<int64_t>(1, h.tlbf.part_len));   // FP32 partial sums
    if (h.smoother_precision == 64 || h.smoother_form == HPLMM_SMOOTHER_INVERSE) {
        // the FP64 contact-grid programs (and the grain inverse) run on the
        // side stream next to the grain and coarse programs, which use tl64's
        // scratch: the side stream needs split-task scratch of its own
        h.d_part_side = h.dalloc<double>(std::max<int64_t>(1, h.tl64.part_len));
    }
    h.d_vtasks = h.upload(h.vtasks, s);
    h.d_vpairs = h.upload(h.vpairs, s);
    h.d_spairs = h.upload(h.spairs, s);
    h.d_rtasks = h.upload(h.rtasks, s);
    h.d_sym_part = h.dalloc<double>(std::max<int64_t>(1, h.sym_part_len));
    h.d_gemv_part = h.dalloc<double>(std::max<int64_t>(1, h.gemv_part_len));
    // arenas and vectors
    h.ar64 = h.dalloc<double>(h.ar64_n);
    // the set-up clears only the envelope tiles of the grain and contact-grid
    // blocks: the rest are zero from here on
    if (!h.zero_g.empty() &&
        hipMemsetAsync(h.ar64 + h.gset.a_base, 0, sizeof(double) * (size_t)h.gset.region, s) != hipSuccess)
        fail(HPLMM_E_HIP, "hipMemsetAsync failed");
    if (!h.zero_c.empty() &&
        hipMemsetAsync(h.ar64 + h.cset.a_base, 0, sizeof(double) * (size_t)h.cset.region, s) != hipSuccess)
        fail(HPLMM_E_HIP, "hipMemsetAsync failed");
    std::vector<double> negi;
    if (h.negi_off >= 0) {
        negi.assign((size_t)TE, 0.0);
        for (int i = 0; i < TS; ++i) negi[(size_t)(i * TS + i)] = -1.0;
        if (hipMemcpyAsync(h.ar64 + h.negi_off, negi.data(), sizeof(double) * TE, hipMemcpyHostToDevice, s) != hipSuccess)
            fail(HPLMM_E_HIP, "hipMemcpyAsync failed");
    }
    if (h.ar32_n) h.ar32 = h.dalloc<float>(h.ar32_n);
    if (h.arbf_n) h.arbf = h.dalloc<uint16_t>(h.arbf_n);
    h.gx = h.dalloc<double>(h.gset.vec_len);
    h.gt = h.dalloc<double>(h.gset.vec_len);
    h.gy = h.dalloc<double>(h.gset.vec_len);
    h.gc_t = h.dalloc<double>(h.gcol_len);
    h.gc_u = h.dalloc<double>(h.gcol_len);
    h.cx = h.dalloc<double>(h.cset.vec_len);
    h.ct = h.dalloc<double>(h.cset.vec_len);
    h.cy = h.dalloc<double>(h.cset.vec_len);
    h.sf = h.dalloc<double>(h.cvec_len);
    h.st = h.dalloc<double>(h.cvec_len);
    h.su = h.dalloc<double>(h.cvec_len);
    if (h.cvec_len > 0) {
        (void)hipMemsetAsync(h.sf, 0, sizeof(double) * (size_t)h.cvec_len, s);
        (void)hipMemsetAsync(h.st, 0, sizeof(double) * (size_t)h.cvec_len, s);
        (void)hipMemsetAsync(h.su, 0, sizeof(double) * (size_t)h.cvec_len, s);
    }
    h.z1 = h.dalloc<double>(h.N);
    h.z2 = h.dalloc<double>(h.N);
    h.r1 = h.dalloc<double>(h.N);
    h.r2 = h.dalloc<double>(h.N);
    h.tmpN = h.dalloc<double>(h.N);
    h.d_flag = h.dalloc<int32_t>(2);
    if (hipStreamSynchronize(s) != hipSuccess) fail(HPLMM_E_HIP, "upload failed");
}

}  // namespace hplmm
