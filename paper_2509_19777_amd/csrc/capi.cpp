// C ABI of libhplmm: plan, numeric set-up, preconditioner application,
// flexible GMRES and introspection.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "../../include/hplmm_debug.h"
#include "../../include/hplmm_surrogate.h"
#include "handle.h"

namespace hplmm {

static void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(HPLMM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Built-in profiler: HIP events recorded on the launch stream around every
// launch of the enabled kernel classes.
struct ProfScope {
    Profiler &p;
    int32_t cls;
    double units;
    hipStream_t s;
    size_t ev = 0;
    bool on;
    ProfScope(Handle &h, int32_t c, double u, hipStream_t st) : p(h.prof), cls(c), units(u), s(st) {
        on = (p.mask >> c) & 1;
        if (!on) return;
        while (p.used + 2 > p.pool.size()) {
            // timing only, read after a device synchronisation: no
            // system-scope fence, whose L2 writeback and invalidation would
            // otherwise land between the kernels being timed
            hipEvent_t e;
            hip_check(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
            p.pool.push_back(e);
        }
        ev = p.used;
        p.used += 2;
        hip_check(hipEventRecord(p.pool[ev], s), "event");
    }
    ~ProfScope() {
        if (!on) return;
        (void)hipEventRecord(p.pool[ev + 1], s);
        p.recs.push_back({cls, ev, units});
    }
};

// part / cnt: split-task scratch (default: the task lists' own)
template <class T>
static void run_program(Handle &h, const TaskLists &tl, T *arena, const std::vector<Launch> &prog, int32_t *flag,
                        hipStream_t s, void *part = nullptr) {
    if (!part) part = tl.d_part;
    for (const Launch &L : prog) {
        switch (L.kind) {
            case LK_DIAG: {
                ProfScope ps(h, PC_DIAG, (double)L.count, s);
                launch_diag<T>(arena, arena, arena, tl.d_diag + L.start, L.count, flag, s);
                break;
            }
            case LK_GEMM: {
                {
                    ProfScope ps(h, PC_TILE_GEMM, L.flops, s);
                    launch_tile_gemm<T>(arena, tl.d_gemm + L.start, tl.d_pairs, L.count, s, (T *)part, false);
                }
                if (L.split) {
                    // the finishing pass, a launch of its own (also for the profiler)
                    ProfScope ps(h, PC_TILE_GEMM, 0.0, s);
                    launch_tile_gemm_finish<T>(arena, tl.d_gemm + L.start, tl.d_pairs, L.count, s, (T *)part);
                }
                break;
            }
            case LK_TRANSPOSE: launch_tile_transpose<T>(arena, arena, tl.d_copy + L.start, L.count, s); break;
        }
    }
}

static void spmv(Handle &h, const double *x, const double *r, double *y, hipStream_t s) {
    ProfScope ps(h, PC_SPMV, h.spmv_bytes + (r ? 24.0 * h.n_nodes : 0.0), s);
    if (h.vop_on)
        launch_spmv_voxel(h.vop, h.vop_xyz, h.vop_K, x, r, y, s);
    else
        launch_spmv(h.sell, x, r, y, s);
}

static void zero(void *p, int64_t bytes, hipStream_t s) {
    if (bytes > 0) hip_check(hipMemsetAsync(p, 0, (size_t)bytes, s), "hipMemsetAsync");
}

struct SgSetup {
    hplmm_sg_net *net;
    double threshold;
    hplmm_sg_stats *stats;
};
static void surrogate_basis(Handle &h, const SgSetup &sg, hipStream_t s);

// Tile contractions with bfloat16 operands and FP32 results.
static void run_bf16_program(Handle &h, const TaskLists &tl, const std::vector<Launch> &prog, hipStream_t s) {
    for (const Launch &L : prog) {
        if (L.kind != LK_GEMM) fail(HPLMM_E_STATE, "internal: bfloat16 programs hold contractions only");
        ProfScope ps(h, PC_TILE_GEMM, L.flops, s);
        launch_tile_gemm_bf16(h.arbf, h.ar32, tl.d_gemm + L.start, tl.d_pairs, L.count, s, (float *)tl.d_part,
                              L.split);
    }
}

// The smoother's symmetric inverse S of a dense set (inverse form), on
// stream s after its factor program.  FP64: S = W^T W from the FP64 W (the
// left operand read transposed).  Reduced precision: W is rounded to the storage
// precision first and S = Wp^T Wp is formed from the rounded values on the
// matrix cores with FP32 accumulation (FP32 operands at 32, bfloat16 operands
// at 16) and kept in FP32 -- the Gram matrix of Wp, positive definite however
// coarse the rounding.
static void form_inverse(Handle &h, const DenseSet &ds, hipStream_t s) {
    if (h.smoother_precision == 64) {
        if (!h.d_part_side) fail(HPLMM_E_STATE, "side-stream split scratch missing");
        run_program<double>(h, h.tl64, h.ar64, ds.inverse_prog, h.d_flag, s, h.d_part_side);
    } else if (h.smoother_precision == 32) {
        launch_convert_f64_f32(h.ar64 + ds.w_base, h.ar32 + ds.low_w_base, ds.region, s);
        run_program<float>(h, h.tl32, h.ar32, ds.inverse_prog, h.d_flag, s);
    } else {
        launch_convert_f64_bf16(h.ar64 + ds.w_base, h.arbf + ds.low_w_base, ds.region, s);
        run_bf16_program(h, h.tlbf, ds.inverse_prog, s);
    }
}

// Contact grids (Eq. 26): blocks, factor and inverse, on stream s; in FP64
// except in the reduced-precision factor form.
static void contact_setup(Handle &h, hipStream_t s) {
    if (h.smoother_precision == 64 || h.smoother_form == HPLMM_SMOOTHER_INVERSE) {
        // FP64 programs beside those on the main stream: never on its scratch
        if (!h.d_part_side) fail(HPLMM_E_STATE, "side-stream split scratch missing");
        if (!h.zero_c.empty())
            launch_zero_runs(h.d_zero_c, (int64_t)h.zero_c.size() / 2, h.ar64, s);
        else
            zero(h.ar64 + h.cset.a_base, sizeof(double) * h.cset.region, s);
        launch_gather_contact_blocks(h.csr, h.cg, h.n_citems, h.ar64, s);
        launch_set_ones(h.d_pad_c, (int64_t)h.pad_ones_c.size(), h.ar64, s);
        run_program<double>(h, h.tl64, h.ar64, h.cset.factor_prog, h.d_flag, s, h.d_part_side);
        if (h.smoother_form == HPLMM_SMOOTHER_INVERSE) form_inverse(h, h.cset, s);
    } else {
        zero(h.ar64 + h.c_stage_base, sizeof(double) * h.cset.region, s);
        launch_gather_contact_blocks(h.csr, h.cg, h.n_citems, h.ar64, s);
        launch_set_ones(h.d_pad_c, (int64_t)h.pad_ones_c.size(), h.ar64, s);
        launch_convert_f64_f32(h.ar64 + h.c_stage_base, h.ar32 + h.cset.a_base, h.cset.region, s);
        run_program<float>(h, h.tl32, h.ar32, h.cset.factor_prog, h.d_flag, s);
        if (h.smoother_precision == 16) {
            launch_convert_f32_bf16(h.ar32 + h.cset.w_base, h.arbf + h.cset.low_w_base, h.cset.region, s);
            launch_convert_f32_bf16(h.ar32 + h.cset.wt_base, h.arbf + h.cset.low_wt_base, h.cset.region, s);
        }
    }
}

// The numeric set-up.  A full set-up (stage 3) runs the contact grids on the
// side stream, forked after the pivot flag is reset and joined at the end,
// beside the grains and the coarse operator on s (disjoint arena regions and
// split-task scratch).
static void numeric_setup(Handle &h, hipStream_t s, int stage = 3, const SgSetup *sg = nullptr) {
    struct Events {
        hipEvent_t e[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
        ~Events() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } evs;
    hipEvent_t *ev = evs.e;
    for (int i = 0; i < 8; ++i) hip_check(hipEventCreate(&ev[i]), "hipEventCreate");
    const int32_t init_flag[2] = {0, 0x7fffffff};
    hip_check(hipMemcpyAsync(h.d_flag, init_flag, sizeof(init_flag), hipMemcpyHostToDevice, s), "flag init");
    hip_check(hipEventRecord(ev[0], s), "event");
    const bool fork = stage >= 3;
    if (fork) {
        if (!h.side) {
            hip_check(hipStreamCreateWithFlags(&h.side, hipStreamNonBlocking), "stream");
            for (auto &e : h.side_ev) hip_check(hipEventCreate(&e), "event");
        }
    }
    // the grains' coupling blocks R (the basis right-hand sides), cleared and
    // gathered on the side stream beside the grain blocks on s
    auto gather_r = [&](hipStream_t st) {
        if (!h.gm_roff.empty()) {
            const int64_t r0 = h.gm_roff[0];
            int64_t rlen = 0;
            for (size_t m = 0; m < h.gm_roff.size(); ++m) rlen += h.gset.nt[m] * h.gm_ntc[m] * TE;
            zero(h.ar64 + r0, sizeof(double) * rlen, st);
        }
        launch_gather_abar(h.csr, h.d_abar, h.n_abar, h.cm, h.gg, h.ar64, st);
    };
    if (fork) {
        hip_check(hipStreamWaitEvent(h.side, ev[0], 0), "fork");
        gather_r(h.side);
        hip_check(hipEventRecord(ev[7], h.side), "event");
    }
    if (fork && h.n_mortar > 0) {
        // the fronts' region is cleared on the side stream, idle until the
        // grains are factored
        zero(h.ar64 + h.mf.a_base, sizeof(double) * h.mf.region, h.side);
        hip_check(hipEventRecord(ev[6], h.side), "event");
    }
    // ---- grains: blocks, factor, inverse, basis (Eqs. 23-24) ----
    if (!h.zero_g.empty())
        launch_zero_runs(h.d_zero_g, (int64_t)h.zero_g.size() / 2, h.ar64, s);
    else
        zero(h.ar64 + h.gset.a_base, sizeof(double) * h.gset.region, s);
    launch_gather_grain_blocks(h.csr, h.gg, h.d_b, h.ar64, s);
    launch_set_ones(h.d_pad_g, (int64_t)h.pad_ones_g.size(), h.ar64, s);
    if (fork)
        hip_check(hipStreamWaitEvent(s, ev[7], 0), "join");
    else
        gather_r(s);
    if (stage < 1) {
        hip_check(hipStreamSynchronize(s), "stage");
        return;
    }
    run_program<double>(h, h.tl64, h.ar64, h.gset.factor_prog, h.d_flag, s);
    hip_check(hipEventRecord(ev[5], s), "event");
    // W = L^-1 of the grains, when not formed in the factorisation's steps,
    // is needed only by the grain inverse (side stream, below), except by the
    // learned basis's exact fallback and in a staged set-up
    const bool w_side = fork && !sg && h.smoother_form == HPLMM_SMOOTHER_INVERSE;
    if (!w_side) run_program<double>(h, h.tl64, h.ar64, h.gset.w_prog, h.d_flag, s);
    // the contact grids start once the grain factorisation is done: its
    // chain of small dependent launches runs best alone, while the grain
    // basis and the coarse factorisation leave room beside them.  With the
    // exact basis they are queued after it, so that queueing their many
    // launches never leaves the main stream idle.
    auto fork_contacts = [&] {
        hip_check(hipStreamWaitEvent(h.side, ev[5], 0), "fork");
        hip_check(hipEventRecord(h.side_ev[0], h.side), "event");
        contact_setup(h, h.side);
        hip_check(hipEventRecord(h.side_ev[1], h.side), "event");
    };
    if (fork && sg) fork_contacts();
    if (stage < 2) {
        hip_check(hipStreamSynchronize(s), "stage");
        return;
    }
    if (sg) {
        surrogate_basis(h, *sg, s);
    } else {
        run_program<double>(h, h.tl64, h.ar64, h.basis_prog, h.d_flag, s);
        // X (by substitution) is read only by the preconditioner's
        // application: beside the coarse operator, ahead of the contact grids
        if (fork) {
            hip_check(hipStreamWaitEvent(h.side, ev[5], 0), "fork");
            run_program<double>(h, h.tl64, h.ar64, h.basis_x_prog, h.d_flag, h.side, h.d_part_side);
        } else {
            run_program<double>(h, h.tl64, h.ar64, h.basis_x_prog, h.d_flag, s);
        }
    }
    if (fork && !sg) fork_contacts();
    if (fork) {
        // the grain inverse S = W^T W (after the rows of W, when those are
        // not formed in the factorisation's steps) follows the contact grids
        // on the side stream, beside the coarse operator on s
        if (h.smoother_form == HPLMM_SMOOTHER_INVERSE) {
            if (!w_side) {
                // W came from the main stream
                hip_check(hipEventRecord(ev[4], s), "event");
                hip_check(hipStreamWaitEvent(h.side, ev[4], 0), "wait");
            }
            hip_check(hipEventRecord(h.side_ev[3], h.side), "event");
            if (w_side) {
                if (!h.d_part_side) fail(HPLMM_E_STATE, "side-stream split scratch missing");
                run_program<double>(h, h.tl64, h.ar64, h.gset.w_prog, h.d_flag, h.side, h.d_part_side);
            }
            form_inverse(h, h.gset, h.side);
        }
        hip_check(hipEventRecord(h.side_ev[2], h.side), "event");
    }
    if (stage < 3) {
        hip_check(hipStreamSynchronize(s), "stage");
        return;
    }
    launch_gather_scalar(h.d_corr_koff, h.n_corr, h.ar64, h.corr_d, s);
    if (h.smoother_form == HPLMM_SMOOTHER_INVERSE) {
        // the smoother reads S, rounded on the side stream
    } else if (h.smoother_precision == 32) {
        launch_convert_f64_f32(h.ar64 + h.gset.w_base, h.ar32 + h.gset.low_w_base, h.gset.region, s);
        launch_convert_f64_f32(h.ar64 + h.gset.wt_base, h.ar32 + h.gset.low_wt_base, h.gset.region, s);
    } else if (h.smoother_precision == 16) {
        launch_convert_f64_bf16(h.ar64 + h.gset.w_base, h.arbf + h.gset.low_w_base, h.gset.region, s);
        launch_convert_f64_bf16(h.ar64 + h.gset.wt_base, h.arbf + h.gset.low_wt_base, h.gset.region, s);
    }
    hip_check(hipEventRecord(ev[1], s), "event");
    // ---- coarse operator P^T A P (Eq. 18) and its factorisation ----
    if (h.n_mortar > 0) {
        // assemble every front, then factor level by level from the leaves,
        // adding each child's update matrix into its parent first
        CoarseMF &mf = h.mf;
        if (fork)
            hip_check(hipStreamWaitEvent(s, ev[6], 0), "wait");
        else
            zero(h.ar64 + mf.a_base, sizeof(double) * mf.region, s);
        launch_coarse_assemble(h.d_pairs, h.n_pairs, h.d_edges, h.d_krefs, h.cm, h.csr.val, h.ar64, h.ar64,
                               h.pair_vals, s);
        launch_set_ones(mf.d_pad, (int64_t)mf.pad_ones.size(), h.ar64, s);
        for (int32_t l = mf.n_levels - 1; l >= 0; --l) {
            const Range r = mf.ext_lvl[(size_t)l];
            launch_extend_add(mf.d_ext + r.start, r.count, mf.d_inv, h.ar64, s);
            run_program<double>(h, h.tl64, h.ar64, mf.factor_prog[(size_t)l], h.d_flag, s);
        }
    }
    hip_check(hipEventRecord(ev[2], s), "event");
    hip_check(hipStreamWaitEvent(s, h.side_ev[2], 0), "join");
    hip_check(hipEventRecord(ev[3], s), "event");
    hip_check(hipGetLastError(), "kernel launch");
    int32_t flag[2];
    hip_check(hipMemcpyAsync(flag, h.d_flag, sizeof(flag), hipMemcpyDeviceToHost, s), "flag copy");
    std::vector<double> cd((size_t)h.n_corr);
    if (h.n_corr)
        hip_check(hipMemcpyAsync(cd.data(), h.corr_d, sizeof(double) * cd.size(), hipMemcpyDeviceToHost, s), "corr copy");
    hip_check(hipStreamSynchronize(s), "set-up");
    // phases: grains [0, 1], contact grids on the side stream, coarse [1, 2];
    // the total is the wall time [0, 3]
    float ms[4];
    hip_check(hipEventElapsedTime(&ms[0], ev[0], ev[1]), "elapsed");
    hip_check(hipEventElapsedTime(&ms[1], h.side_ev[0], h.side_ev[1]), "elapsed");
    hip_check(hipEventElapsedTime(&ms[2], ev[1], ev[2]), "elapsed");
    hip_check(hipEventElapsedTime(&ms[3], ev[0], ev[3]), "elapsed");
    for (int i = 0; i < 4; ++i) h.t_setup_ms[i] = ms[i];
    // the paper's split of the set-up: T_ML, the smoother's local
    // factorisations (grain factors, contact grids, the grain inverse S), and
    // T_MG, the coarse space (basis, coarse operator and its factor); the
    // contact grids and S run beside the others, so T_ML + T_MG exceeds the
    // wall time
    float f_ms = 0.f, s_ms = 0.f, b_ms = 0.f;
    hip_check(hipEventElapsedTime(&f_ms, ev[0], ev[5]), "elapsed");
    hip_check(hipEventElapsedTime(&b_ms, ev[5], ev[1]), "elapsed");
    if (h.smoother_form == HPLMM_SMOOTHER_INVERSE)
        hip_check(hipEventElapsedTime(&s_ms, h.side_ev[3], h.side_ev[2]), "elapsed");
    h.t_ml_ms = (double)f_ms + ms[1] + s_ms;
    h.t_mg_ms = (double)b_ms + ms[2];
    if (flag[0]) {
        const int set = flag[1] >> 26, m = flag[1] & ((1 << 26) - 1);
        const char *names[3] = {"grain", "contact-grid", "coarse"};
        fail(HPLMM_E_NOT_SPD, std::string("non-positive Cholesky pivot in ") + names[set < 3 ? set : 0] +
                                  " block " + std::to_string(m));
    }
    for (size_t j = 0; j < cd.size(); ++j)
        if (!(cd[j] > 0.0)) fail(HPLMM_E_SINGULAR_COARSE, "coarse correction pivot <= 0 for correction " + std::to_string(j));
    h.ready = true;
}

// ---- learned-basis set-up ------------------------------------------------------------
// Upload a task list built on the host into the handle's surrogate scratch
// buffers (grown on demand) and run its launches.
static void run_host_program(Handle &h, TaskLists &tl, std::vector<Launch> &prog, hipStream_t s, int64_t z_lo = 0,
                             int64_t z_hi = 0) {
    if (prog.empty()) return;
    // every tile must lie in the arena or in the scratch range [z_lo, z_hi)
    auto ok = [&](int64_t o) { return (o >= 0 && o + TE <= h.ar64_n) || (o >= z_lo && o + TE <= z_hi); };
    for (const GemmTask &t : tl.gemm) {
        if (!ok(t.c_off) || (t.post_off >= 0 && !ok(t.post_off)) || t.pair_start < 0 ||
            (size_t)t.pair_start + (size_t)t.pair_count > tl.pairs.size())
            fail(HPLMM_E_ARG, "internal: surrogate task out of range");
    }
    for (const GemmPair &p : tl.pairs)
        if (!ok(p.a_off) || !ok(p.b_off)) fail(HPLMM_E_ARG, "internal: surrogate operand out of range");
    for (const CopyTask &c : tl.copy)
        if (!ok(c.src_off) || !ok(c.dst_off)) fail(HPLMM_E_ARG, "internal: surrogate copy out of range");
    for (const Launch &L : prog) {
        const size_t n = L.kind == LK_GEMM ? tl.gemm.size() : tl.copy.size();
        if (L.kind == LK_DIAG || L.start < 0 || (size_t)(L.start + L.count) > n)
            fail(HPLMM_E_ARG, "internal: surrogate launch out of range");
    }
    fill_flops(prog, tl);
    auto up = [&](Handle::Scratch &sc, const void *src, size_t bytes) {
        void *d = sc.get(std::max<size_t>(bytes, 16));
        if (bytes) hip_check(hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, s), "copy tasks");
        return d;
    };
    TaskLists dev;
    dev.d_gemm = (GemmTask *)up(h.sg_tasks, tl.gemm.data(), sizeof(GemmTask) * tl.gemm.size());
    dev.d_pairs = (GemmPair *)up(h.sg_pairs, tl.pairs.data(), sizeof(GemmPair) * tl.pairs.size());
    dev.d_copy = (CopyTask *)up(h.sg_copy, tl.copy.data(), sizeof(CopyTask) * tl.copy.size());
    run_program<double>(h, dev, h.ar64, prog, h.d_flag, s);
    // the pageable task vectors must stay alive until the copies are done
    hip_check(hipStreamSynchronize(s), "sync");
}

// Shape vectors of the grains from the network where they pass the residual
// check, exact elsewhere.  On entry the grain factors (L in place of A, W,
// W^T) are done and R holds [-Abar | b].  Regions: R0 = R saved in the XT
// region, B~ (predictions) in R, T = L^T B~ in Y, Z = R0 - L T = -(A B~ + Abar)
// in scratch.  A grain is accepted when it has no correction column and
// |Z e_k| <= threshold |R0 e_k| for all its columns; its Galerkin block is
// K = B~^T A B~ - B~^T Abar - Abar^T B~ = T^T T + Z^T B~ + B~^T Z.  Other grains
// get R restored and the exact basis program.
static void surrogate_basis(Handle &h, const SgSetup &sg, hipStream_t s) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    const int64_t nG = (int64_t)h.gm_grain.size();
    if (nG == 0) return;
    if (!sg_net_is_basis_net(sg.net)) fail(HPLMM_E_ARG, "the network must map 4 input channels to 9 outputs");
    sg_build_sample_tables(h, s);
    int64_t rlen = 0;
    for (int64_t m = 0; m < nG; ++m) rlen += h.gset.nt[m] * h.gm_ntc[(size_t)m] * TE;
    const int64_t r_base = h.gm_roff[0], xt_base = h.gm_xtoff[0];
    double *A = h.ar64;
    hip_check(hipMemcpyAsync(A + xt_base, A + r_base, sizeof(double) * (size_t)rlen, hipMemcpyDeviceToDevice, s),
              "save R0");
    // inference, in batches of the network's size
    const int32_t nb = sg_net_max_batch(sg.net);
    float *xb = (float *)h.sg_x.get(sizeof(float) * (size_t)nb * sg::P * 4);
    float *yb = (float *)h.sg_y.get(sizeof(float) * (size_t)nb * sg::P * 9);
    for (int64_t f = 0; f < h.sg_total; f += nb) {
        const int32_t cnt = (int32_t)std::min<int64_t>(nb, h.sg_total - f);
        sg::launch_fill_samples(h.sg_args, f, cnt, xb, nullptr, s);
        sg_net_forward(sg.net, xb, cnt, yb, s);
        sg::launch_scatter_pred(h.sg_args, f, cnt, yb, A, s);
    }
    hip_check(hipGetLastError(), "inference launch");
    hip_check(hipStreamSynchronize(s), "sync");
    const auto t1 = clk::now();
    // residual check: T = L^T B~, Z = R0 - L T (Z starts as a copy of R0)
    double *Z = (double *)h.sg_z.get(sizeof(double) * (size_t)rlen);
    const int64_t z_shift = (int64_t)(Z - A);   // Z's offset as seen from the arena base
    hip_check(hipMemcpyAsync(Z, A + xt_base, sizeof(double) * (size_t)rlen, hipMemcpyDeviceToDevice, s), "copy R0");
    auto Lt = [&](int64_t m, int64_t I, int64_t J) { return h.gset.a_base + h.gset.rel[m] + tri_index(I, J) * TE; };
    auto Rt = [&](int64_t base, int64_t m, int64_t I, int64_t C) { return base + (C * h.gset.nt[m] + I) * TE; };
    {
        TaskLists tl;
        std::vector<Launch> prog;
        Launch l1{LK_GEMM, 0, 0};
        for (int64_t m = 0; m < nG; ++m)
            for (int64_t C = 0; C < h.gm_ntc[(size_t)m]; ++C)
                for (int64_t I = 0; I < h.gset.nt[m]; ++I) {
                    tl.gemm.push_back({Rt(h.gm_ytoff[(size_t)m], m, I, C), -1, (int32_t)tl.pairs.size(),
                                       (int32_t)(h.gset.nt[m] - I), GF_TRANS_A, 0});
                    for (int64_t J = I; J < h.gset.nt[m]; ++J)
                        tl.pairs.push_back({Lt(m, J, I), Rt(h.gm_roff[(size_t)m], m, J, C)});
                }
        l1.count = (int64_t)tl.gemm.size();
        prog.push_back(l1);
        Launch l2{LK_GEMM, (int64_t)tl.gemm.size(), 0};
        for (int64_t m = 0; m < nG; ++m)
            for (int64_t C = 0; C < h.gm_ntc[(size_t)m]; ++C)
                for (int64_t I = 0; I < h.gset.nt[m]; ++I) {
                    tl.gemm.push_back({Rt(z_shift + h.gm_roff[(size_t)m] - r_base, m, I, C), -1,
                                       (int32_t)tl.pairs.size(), (int32_t)(I + 1), GF_ACCUM | GF_NEGATE, 0});
                    for (int64_t J = 0; J <= I; ++J)
                        tl.pairs.push_back({Lt(m, I, J), Rt(h.gm_ytoff[(size_t)m], m, J, C)});
                }
        l2.count = (int64_t)tl.gemm.size() - l2.start;
        prog.push_back(l2);
        run_host_program(h, tl, prog, s, z_shift, z_shift + rlen);
    }
    // column norms of R0 and Z
    std::vector<int64_t> off0, offz, cofs;
    std::vector<int32_t> ntv, ctv, ncv;
    for (int64_t m = 0; m < nG; ++m)
        for (int64_t C = 0; C < h.gm_ntc[(size_t)m]; ++C) {
            off0.push_back(h.gm_xtoff[(size_t)m]);
            offz.push_back(z_shift + h.gm_roff[(size_t)m] - r_base);
            ntv.push_back((int32_t)h.gset.nt[m]);
            ctv.push_back((int32_t)C);
            cofs.push_back(h.gm_coff[(size_t)m]);
            ncv.push_back(h.gm_ncol[(size_t)m]);
        }
    const int64_t nt_tasks = (int64_t)off0.size();
    const size_t meta_bytes = sizeof(int64_t) * 3 * (size_t)nt_tasks + sizeof(int32_t) * 3 * (size_t)nt_tasks;
    char *meta = (char *)h.sg_meta.get(meta_bytes);
    int64_t *d_off0 = (int64_t *)meta, *d_offz = d_off0 + nt_tasks, *d_cofs = d_offz + nt_tasks;
    int32_t *d_nt = (int32_t *)(d_cofs + nt_tasks), *d_ct = d_nt + nt_tasks, *d_nc = d_ct + nt_tasks;
    hip_check(hipMemcpyAsync(d_off0, off0.data(), 8 * off0.size(), hipMemcpyHostToDevice, s), "copy");
    hip_check(hipMemcpyAsync(d_offz, offz.data(), 8 * offz.size(), hipMemcpyHostToDevice, s), "copy");
    hip_check(hipMemcpyAsync(d_cofs, cofs.data(), 8 * cofs.size(), hipMemcpyHostToDevice, s), "copy");
    hip_check(hipMemcpyAsync(d_nt, ntv.data(), 4 * ntv.size(), hipMemcpyHostToDevice, s), "copy");
    hip_check(hipMemcpyAsync(d_ct, ctv.data(), 4 * ctv.size(), hipMemcpyHostToDevice, s), "copy");
    hip_check(hipMemcpyAsync(d_nc, ncv.data(), 4 * ncv.size(), hipMemcpyHostToDevice, s), "copy");
    double *nrm = (double *)h.sg_norms.get(sizeof(double) * 2 * (size_t)std::max<int64_t>(1, h.gcol_len));
    sg::launch_col_norms(A, d_off0, d_nt, d_ct, d_cofs, d_nc, nt_tasks, nrm, s);
    sg::launch_col_norms(A, d_offz, d_nt, d_ct, d_cofs, d_nc, nt_tasks, nrm + h.gcol_len, s);
    std::vector<double> hn(2 * (size_t)h.gcol_len);
    hip_check(hipMemcpyAsync(hn.data(), nrm, sizeof(double) * hn.size(), hipMemcpyDeviceToHost, s), "copy norms");
    hip_check(hipStreamSynchronize(s), "sync");
    const auto t2 = clk::now();
    // acceptance
    std::vector<int64_t> exact, accepted;
    std::vector<double> ratios;
    double max_acc = 0.0;
    for (int64_t m = 0; m < nG; ++m) {
        const bool loaded = h.gm_corr[(size_t)m] >= 0;
        double worst = 0.0;
        for (int32_t j = 0; j < h.gm_k[(size_t)m]; ++j) {
            const double a0 = hn[(size_t)(h.gm_coff[(size_t)m] + j)], z = hn[(size_t)(h.gcol_len + h.gm_coff[(size_t)m] + j)];
            const double r = a0 > 0.0 ? std::sqrt(z / a0) : (z > 0.0 ? INFINITY : 0.0);
            ratios.push_back(r);
            worst = std::max(worst, r);
        }
        if (!loaded && worst <= sg.threshold) {
            accepted.push_back(m);
            max_acc = std::max(max_acc, worst);
        } else {
            exact.push_back(m);
        }
    }
    // exact grains: restore R, exact basis; accepted grains: K = T^T T + Z^T B~ + B~^T Z
    for (int64_t m : exact) {
        const int64_t len = h.gset.nt[m] * h.gm_ntc[(size_t)m] * TE;
        hip_check(hipMemcpyAsync(A + h.gm_roff[(size_t)m], A + h.gm_xtoff[(size_t)m], sizeof(double) * (size_t)len,
                                 hipMemcpyDeviceToDevice, s),
                  "restore R");
    }
    {
        TaskLists tl;
        std::vector<Launch> prog;
        append_basis_program(h, tl, exact, prog, BP_Y | BP_X | BP_K);
        for (int pass = 0; pass < 3; ++pass) {
            Launch L{LK_GEMM, (int64_t)tl.gemm.size(), 0};
            for (int64_t m : accepted) {
                const int64_t zb = z_shift + h.gm_roff[(size_t)m] - r_base;
                for (int64_t C1 = 0; C1 < h.gm_ntc[(size_t)m]; ++C1)
                    for (int64_t C2 = 0; C2 <= C1; ++C2) {
                        tl.gemm.push_back({h.gm_koff[(size_t)m] + tri_index(C1, C2) * TE, -1, (int32_t)tl.pairs.size(),
                                           (int32_t)h.gset.nt[m], pass == 0 ? GF_TRANS_A : (GF_TRANS_A | GF_ACCUM), 0});
                        for (int64_t I = 0; I < h.gset.nt[m]; ++I) {
                            if (pass == 0)
                                tl.pairs.push_back({Rt(h.gm_ytoff[(size_t)m], m, I, C1), Rt(h.gm_ytoff[(size_t)m], m, I, C2)});
                            else if (pass == 1)
                                tl.pairs.push_back({Rt(zb, m, I, C1), Rt(h.gm_roff[(size_t)m], m, I, C2)});
                            else
                                tl.pairs.push_back({Rt(h.gm_roff[(size_t)m], m, I, C1), Rt(zb, m, I, C2)});
                        }
                    }
            }
            L.count = (int64_t)tl.gemm.size() - L.start;
            if (L.count) prog.push_back(L);
        }
        std::vector<int64_t> all((size_t)nG);
        for (int64_t m = 0; m < nG; ++m) all[(size_t)m] = m;
        append_basis_program(h, tl, all, prog, BP_XT);
        run_host_program(h, tl, prog, s, z_shift, z_shift + rlen);
    }
    const auto t3 = clk::now();
    if (sg.stats) {
        hplmm_sg_stats &st = *sg.stats;
        st.grains = (int32_t)nG;
        st.accepted = (int32_t)accepted.size();
        st.fallback = (int32_t)exact.size();
        st.loaded = 0;
        for (int64_t m = 0; m < nG; ++m) st.loaded += h.gm_corr[(size_t)m] >= 0;
        st.max_residual_accepted = max_acc;
        std::vector<double> r = ratios;
        if (!r.empty()) {
            std::nth_element(r.begin(), r.begin() + (long)(r.size() / 2), r.end());
            st.median_residual = r[r.size() / 2];
        } else {
            st.median_residual = 0.0;
        }
        auto ms = [](clk::time_point a, clk::time_point b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
        st.t_infer_ms = ms(t0, t1);
        st.t_check_ms = ms(t1, t2);
        st.t_basis_ms = ms(t2, t3);
    }
}

static void launch_set(Handle &h, const Range &r, bool smoother_low, const double *x, double *y, hipStream_t s) {
    const GemvTask *t = h.d_vtasks + r.start;
    if (r.sym) {
        // S is kept in FP64 at full precision and in FP32 otherwise
        if (h.smoother_precision == 64)
            launch_sym_gemv<double>(h.ar64, x, y, t, h.d_spairs, r.count, h.d_sym_part, r.waves, s);
        else
            launch_sym_gemv<float>(h.ar32, x, y, t, h.d_spairs, r.count, h.d_sym_part, r.waves, s);
    } else if (!smoother_low || h.smoother_precision == 64)
        launch_gemv<double>(h.ar64, x, y, t, h.d_vpairs, r.count, s, nullptr, r.waves);
    else if (h.smoother_precision == 32)
        launch_gemv<float>(h.ar32, x, y, t, h.d_vpairs, r.count, s, nullptr, r.waves);
    else
        launch_gemv<uint16_t>(h.arbf, x, y, t, h.d_vpairs, r.count, s, nullptr, r.waves);
}

static void gemv_set(Handle &h, const Range &r, bool smoother_low, const double *x, double *y, hipStream_t s,
                     int32_t cls = PC_GEMV_SMOOTH) {
    if (r.count == 0) return;
    ProfScope ps(h, cls, r.bytes, s);
    launch_set(h, r, smoother_low, x, y, s);
}

// Front sweeps: few long rows per launch, split over many work-groups.
// Split rows use the handle's partial-sum buffer, or the static one
// (split_part, set by the allocation-free entry point), and a reduction
// launch finishes them.
static void gemv_front(Handle &h, const Range &r, hipStream_t s) {
    if (r.count == 0) return;
    double *part = h.split_part ? h.split_part : h.d_gemv_part;
    launch_gemv<double>(h.ar64, h.mf.V, h.mf.V, h.d_vtasks + r.start, h.d_vpairs, r.count, s, h.mf.V, r.waves, part);
    if (r.split) launch_gemv_split_reduce(h.d_vtasks + r.start, r.count, part, h.mf.V, h.mf.V, s);
}

// u = S^-1 f for the mortar block of the coarse operator with the
// multifrontal factor: forward sweep from the leaves (y = W11 w and
// w_b -= G w with G = L21 W11, w_b then added into the parent), backward sweep
// from the root (x = W11^T y - G^T x_b, x_b taken from the parent).
static void coarse_solve(Handle &h, const double *f, double *u, hipStream_t s) {
    CoarseMF &mf = h.mf;
    if (mf.n_fronts == 0) return;
    ProfScope ps(h, PC_GEMV_COARSE, 2.0 * mf.factor_bytes, s);
    launch_gather(mf.d_init_map, f, mf.WV, mf.vec_len, s);
    for (int32_t l = mf.n_levels - 1; l >= 0; --l) {
        const Range ve = mf.vec_ext[(size_t)l];
        launch_gather_add(mf.d_va_dst + ve.start, mf.d_va_ptr + ve.start, mf.d_va_src, ve.count, mf.WV, mf.WV, s);
        gemv_front(h, mf.fwd[(size_t)l], s);
    }
    for (int32_t l = 0; l < mf.n_levels; ++l) {
        const Range cp = mf.bwd_copy[(size_t)l];
        launch_copy_idx(mf.d_cp_dst + cp.start, mf.d_cp_src + cp.start, cp.count, mf.XV, mf.XV, s);
        gemv_front(h, mf.bwd[(size_t)l], s);
    }
    launch_copy_idx(mf.d_out_dst, mf.d_out_src, (int64_t)mf.out_dst.size(), mf.XV, u, s);
}

// y = A^-1 x for every matrix of a dense set: y = W^T (W x) (factor form,
// reduced precision applies to the stored operators) or y = S x, with the
// transposed products of the tiles below the diagonal summed into y after the
// pass (inverse form).
static void set_solve(Handle &h, DenseSet &ds, const double *x, double *t, double *y, hipStream_t s) {
    if (h.smoother_form == HPLMM_SMOOTHER_INVERSE) {
        gemv_set(h, ds.gemv_S, false, x, y, s);
        if (ds.red_S.count) {
            ProfScope ps(h, PC_SMOOTH_REDUCE, ds.red_S.bytes, s);
            launch_sym_reduce(h.d_rtasks + ds.red_S.start, ds.red_S.count, h.d_sym_part, y, s);
        }
        return;
    }
    const bool low = h.smoother_precision != 64;
    gemv_set(h, ds.gemv_W, low, x, t, s);
    gemv_set(h, ds.gemv_Wt, low, t, y, s);
}

// Contact-grid smoother (Eq. 26).
static void contact_solve(Handle &h, const double *rr, hipStream_t s) {
    launch_gather(h.d_c_slot_dof, rr, h.cx, h.cset.vec_len, s);
    set_solve(h, h.cset, h.cx, h.ct, h.cy, s);
}

static void grain_solve(Handle &h, const double *rr, hipStream_t s) {
    launch_gather(h.d_g_slot_dof, rr, h.gx, h.gset.vec_len, s);
    set_solve(h, h.gset, h.gx, h.gt, h.gy, s);
}

// z1 = M_G^-1 r = P^ (P^T A P^)^-1 P^T r   (Eq. 18)
static void coarse_apply(Handle &h, const double *r, double *z, hipStream_t s) {
    launch_gather(h.d_g_slot_dof, r, h.gx, h.gset.vec_len, s);
    gemv_set(h, h.gemv_XT, false, h.gx, h.gc_t, s, PC_GEMV_BASIS);
    launch_coarse_rhs(h.cm, r, h.gc_t, h.sf, s);
    coarse_solve(h, h.sf, h.su, s);
    launch_corr_solve(h.cm, h.sf, h.su, s);
    launch_gather(h.d_gcol_upos, h.su, h.gc_u, h.gcol_len, s);
    gemv_set(h, h.gemv_X, false, h.gc_u, h.gy, s, PC_GEMV_BASIS);
    launch_prolong_nodes(h.cm, h.n_nodes, h.d_g_dof_slot, h.gy, h.su, z, s);
}

void apply_op(Handle &h, int32_t which, const double *r, double *z, hipStream_t s) {
    const int64_t N = h.N;
    ProfScope ps(h, PC_APPLY, which == 0 ? h.apply_bytes : 0.0, s);
    switch (which) {
        case 1:
            coarse_apply(h, r, z, s);
            return;
        case 3:
            contact_solve(h, r, s);
            launch_combine(N, nullptr, nullptr, nullptr, h.d_c_dof_ptr, h.d_c_dof_slot, h.cy, z, s);
            return;
        case 4:
            grain_solve(h, r, s);
            launch_combine(N, nullptr, h.d_g_dof_slot, h.gy, nullptr, nullptr, nullptr, z, s);
            return;
        case 2: {
            // M_CG^-1 r = M_zeta^-1 r + M_g^-1 (r - A M_zeta^-1 r)   (Eq. 25)
            contact_solve(h, r, s);
            launch_combine(N, nullptr, nullptr, nullptr, h.d_c_dof_ptr, h.d_c_dof_slot, h.cy, h.z2, s);
            spmv(h, h.z2, r, h.r2, s);
            grain_solve(h, h.r2, s);
            launch_combine(N, h.z2, h.d_g_dof_slot, h.gy, nullptr, nullptr, nullptr, z, s);
            return;
        }
        case 0: {
            // M^-1 r = M_G^-1 r + M_CG^-1 (r - A M_G^-1 r)   (Eq. 16)
            coarse_apply(h, r, h.z1, s);
            spmv(h, h.z1, r, h.r1, s);
            contact_solve(h, h.r1, s);
            launch_combine(N, nullptr, nullptr, nullptr, h.d_c_dof_ptr, h.d_c_dof_slot, h.cy, h.z2, s);
            spmv(h, h.z2, h.r1, h.r2, s);
            grain_solve(h, h.r2, s);
            launch_combine(N, h.z1, h.d_g_dof_slot, h.gy, h.d_c_dof_ptr, h.d_c_dof_slot, h.cy, z, s);
            return;
        }
        default:
            fail(HPLMM_E_ARG, "which must be 0..4");
    }
}

// ---- flexible GMRES (right preconditioning) --------------------------------------
static void ensure_krylov(Handle &h, int32_t restart) {
    if (h.kr_restart >= restart) return;
    h.kr_restart = restart;
    h.V = h.dalloc<double>((int64_t)(restart + 1) * h.N);
    h.Z = h.dalloc<double>((int64_t)restart * h.N);
    h.w = h.dalloc<double>(h.N);
    h.kr_blocks = multidot_blocks(h.N);
    h.part = h.dalloc<double>((int64_t)h.kr_blocks * (restart + 2));
    h.hbuf = h.dalloc<double>(restart + 4);
    h.h2 = h.dalloc<double>(restart + 4);
    h.ydev = h.dalloc<double>(restart + 4);
    if (h.hcol_host) {
        (void)hipHostFree(h.hcol_host);
        h.hcol_host = nullptr;
    }
    hip_check(hipHostMalloc((void **)&h.hcol_host, sizeof(double) * 2 * (size_t)(restart + 4), hipHostMallocDefault),
              "hipHostMalloc");
    for (hipEvent_t &e : h.hcol_ev)
        if (!e) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
}

static double device_dot(Handle &h, const double *a, const double *b, double *dst, hipStream_t s) {
    launch_kr_pass(nullptr, 0, 0, nullptr, b, nullptr, h.N, a, 0, 1, h.part, s);
    launch_kr_reduce(h.part, h.kr_blocks, 1, dst, nullptr, s);
    double v;
    hip_check(hipMemcpyAsync(&v, dst, sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    hip_check(hipStreamSynchronize(s), "sync");
    return v;
}

// One Arnoldi step j of FGMRES: z_j = M^-1 v_j, w = A z_j, classical
// Gram-Schmidt twice (h = V^T w; w -= V h and h2 = V^T w in one pass; w -= V h2
// into v_{j+1} with |w|^2 in one pass; h += h2), v_{j+1} normalised.  Kernel
// launches only, so the step can be captured into a graph.
static void arnoldi_step(Handle &h, int32_t j, hipStream_t s) {
    const int64_t N = h.N;
    double *vj = h.V + (int64_t)j * N, *zj = h.Z + (int64_t)j * N;
    apply_op(h, 0, vj, zj, s);
    spmv(h, zj, nullptr, h.w, s);
    const int32_t k = j + 1;
    double *vn = h.V + (int64_t)(j + 1) * N;
    launch_kr_pass(nullptr, 0, 0, nullptr, h.w, nullptr, N, h.V, N, k, h.part, s);
    launch_kr_reduce(h.part, h.kr_blocks, k, h.hbuf, nullptr, s);
    launch_kr_pass(h.V, N, k, h.hbuf, h.w, h.w, N, h.V, N, k, h.part, s);
    launch_kr_reduce(h.part, h.kr_blocks, k, h.h2, h.hbuf, s);
    launch_kr_pass(h.V, N, k, h.h2, h.w, vn, N, nullptr, 0, 1, h.part, s);
    launch_kr_reduce(h.part, h.kr_blocks, 1, h.hbuf + j + 1, nullptr, s);
    launch_normalize(vn, h.hbuf + j + 1, vn, N, s);
}

// The residual estimate must be at least this many times the tolerance for
// the next Arnoldi step to be queued before the current one is read: a single
// step of this solver has not dropped it by more than about 2x here, so the
// extra step at convergence practically never happens.
constexpr double LOOKAHEAD_MARGIN = 50.0;

static hplmm_status gmres(Handle &h, const double *b, double *x, double rtol, int32_t m, int32_t maxit,
                          int32_t fixed, hplmm_solve_info *info, hipStream_t s) {
    ensure_krylov(h, m);
    const int64_t N = h.N;
    // graphs of the Arnoldi steps, captured on an internal stream (the caller's
    // may be the null stream, which cannot be captured) and launched on the
    // caller's; only while the profiler times no solve-phase class (its events
    // are recorded per launch; the set-up classes 0 and 1 are not in the graphs)
    const bool graphs = h.use_graphs && (h.prof.mask & ~((1 << PC_TILE_GEMM) | (1 << PC_DIAG))) == 0;
    if (graphs) {
        if (!h.gstream) {
            hip_check(hipStreamCreateWithFlags(&h.gstream, hipStreamNonBlocking), "stream");
        }
        if (h.graph_key_V != h.V || (int32_t)h.arnoldi_graphs.size() < m) {
            h.drop_graphs();
            h.arnoldi_graphs.assign((size_t)h.kr_restart, nullptr);
            h.graph_key_V = h.V;
        }
    }
    const double bnorm = std::sqrt(device_dot(h, b, b, h.hbuf, s));
    std::vector<double> hist;
    int32_t it = 0;
    double rel = 0.0;
    bool conv = false;
    const int32_t limit = fixed > 0 ? fixed : maxit;
    if (bnorm == 0.0) {
        hip_check(hipMemsetAsync(x, 0, sizeof(double) * (size_t)N, s), "memset");
        conv = true;
    }
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hv(m + 2);
    while (!conv && it < limit) {
        spmv(h, x, b, h.V, s);       // r0 = b - A x
        const double beta = std::sqrt(device_dot(h, h.V, h.V, h.hbuf, s));
        rel = beta / bnorm;
        if (!std::isfinite(beta)) fail(HPLMM_E_NONFINITE, "non-finite residual");
        if (fixed <= 0 && rel < rtol) {
            conv = true;
            break;
        }
        launch_normalize(h.V, h.hbuf, h.V, N, s);
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        // Step j's kernels are followed on the stream by the copy of its
        // Hessenberg column to a pinned slot and an event.  While the residual
        // estimate is far above the tolerance, step j + 1 (which needs only
        // device data: v_{j+1} is normalised on the device) is queued before
        // the host waits for step j's column, so the host's Givens work and the
        // launch latency hide behind step j + 1.  If step j then converges,
        // the queued step was extra work whose results are never read.
        auto queue_step = [&](int32_t jj) {
            if (graphs) {
                hipGraphExec_t &ge = h.arnoldi_graphs[(size_t)jj];
                if (!ge) {
                    hipGraph_t g = nullptr;
                    hip_check(hipStreamBeginCapture(h.gstream, hipStreamCaptureModeThreadLocal), "begin capture");
                    try {
                        arnoldi_step(h, jj, h.gstream);
                    } catch (...) {
                        // leave the stream out of capture mode before reporting
                        if (hipStreamEndCapture(h.gstream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
                        throw;
                    }
                    hip_check(hipStreamEndCapture(h.gstream, &g), "end capture");
                    const hipError_t e = hipGraphInstantiateWithFlags(&ge, g, 0);
                    (void)hipGraphDestroy(g);
                    hip_check(e, "graph instantiate");
                }
                hip_check(hipGraphLaunch(ge, s), "graph launch");
            } else {
                arnoldi_step(h, jj, s);
            }
            double *slot = h.hcol_host + (size_t)(jj & 1) * (size_t)(m + 4);
            hip_check(hipMemcpyAsync(slot, h.hbuf, sizeof(double) * (size_t)(jj + 2), hipMemcpyDeviceToHost, s),
                      "copy h");
            hip_check(hipEventRecord(h.hcol_ev[jj & 1], s), "event");
        };
        int32_t j = 0;
        bool queued = false;   // step j already queued
        for (; j < m && it < limit; ++j) {
            if (!queued) queue_step(j);
            // look ahead while a one-step drop to the tolerance is out of reach
            queued = j + 1 < m && it + 1 < limit && (fixed > 0 || std::fabs(g[j]) / bnorm > LOOKAHEAD_MARGIN * rtol);
            if (queued) queue_step(j + 1);
            hip_check(hipEventSynchronize(h.hcol_ev[j & 1]), "step");
            const double *slot = h.hcol_host + (size_t)(j & 1) * (size_t)(m + 4);
            for (int32_t i = 0; i <= j + 1; ++i) hv[(size_t)i] = slot[i];
            hv[(size_t)j + 1] = std::sqrt(hv[(size_t)j + 1]);
            for (int32_t i = 0; i <= j + 1; ++i)
                if (!std::isfinite(hv[(size_t)i])) fail(HPLMM_E_NONFINITE, "non-finite Arnoldi coefficient");
            double *col = &H[(size_t)j * (m + 1)];
            for (int32_t i = 0; i <= j + 1; ++i) col[i] = hv[(size_t)i];
            for (int32_t i = 0; i < j; ++i) {
                const double t = cs[i] * col[i] + sn[i] * col[i + 1];
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
                col[i] = t;
            }
            const double d = std::hypot(col[j], col[j + 1]);
            cs[j] = col[j] / d;
            sn[j] = col[j + 1] / d;
            col[j] = d;
            col[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            hist.push_back(std::fabs(g[j + 1]) / bnorm);
            if (fixed <= 0 && std::fabs(g[j + 1]) / bnorm < rtol) {
                ++j;
                break;
            }
        }
        const int32_t k = j;
        std::vector<double> y(k);
        for (int32_t i = k - 1; i >= 0; --i) {
            double t = g[i];
            for (int32_t l = i + 1; l < k; ++l) t -= H[(size_t)l * (m + 1) + i] * y[l];
            y[i] = t / H[(size_t)i * (m + 1) + i];
        }
        hip_check(hipMemcpyAsync(h.ydev, y.data(), sizeof(double) * (size_t)k, hipMemcpyHostToDevice, s), "copy y");
        launch_add_combination(h.Z, N, k, h.ydev, x, N, s);
        spmv(h, x, b, h.w, s);
        rel = std::sqrt(device_dot(h, h.w, h.w, h.hbuf, s)) / bnorm;
        if (fixed <= 0 && rel < rtol) conv = true;
    }
    if (info) {
        info->iters = it;
        info->rel_res_true = rel;
        info->res_hist_len = 0;
        if (info->res_hist && info->res_hist_cap > 0) {
            const int32_t n = std::min<int32_t>(info->res_hist_cap, (int32_t)hist.size());
            std::memcpy(info->res_hist, hist.data(), sizeof(double) * (size_t)n);
            info->res_hist_len = n;
        }
    }
    if (fixed > 0) return HPLMM_OK;
    return conv ? HPLMM_OK : HPLMM_NOT_CONVERGED;
}

}  // namespace hplmm

using namespace hplmm;

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" hplmm_status hplmm_plan(const hplmm_system *sys, const hplmm_partition *part, const hplmm_mortar *mortar,
                                   const hplmm_options *opt, void *stream, hplmm_handle **out) {
    return guarded([&]() -> hplmm_status {
        if (!out) fail(HPLMM_E_ARG, "out is NULL");
        *out = nullptr;
        if (!sys || !part || !mortar) fail(HPLMM_E_ARG, "NULL argument");
        hplmm_options o{64, 0};
        if (opt) o = *opt;
        int dev = 0;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        auto *hh = new hplmm_handle();
        try {
            hh->h.device = dev;
            build_plan(hh->h, *sys, *part, *mortar, o, as_stream(stream), false);
            (void)static_scratch_address(dev);   // the allocation-free entry point's buffer on this device
        } catch (...) {
            delete hh;
            throw;
        }
        *out = hh;
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_plan_check(const hplmm_system *sys, const hplmm_partition *part,
                                         const hplmm_mortar *mortar, const hplmm_options *opt, int64_t *sizes) {
    return guarded([&]() -> hplmm_status {
        if (!sys || !part || !mortar) fail(HPLMM_E_ARG, "NULL argument");
        hplmm_options o{64, 0};
        if (opt) o = *opt;
        Handle h;
        build_plan(h, *sys, *part, *mortar, o, nullptr, true);
        if (sizes) {
            int64_t mx_f = 0;
            for (int32_t t = 0; t < h.mf.n_fronts; ++t) mx_f = std::max(mx_f, h.mf.d[(size_t)t] + h.mf.u[(size_t)t]);
            int64_t v[16] = {h.n_nodes, h.nnzb, h.n_grains, h.n_ifaces, h.n_contacts, h.n_mortar, h.n_corr,
                             h.n_coarse, (int64_t)h.gset.n.size(), h.ar64_n, h.ar32_n, h.arbf_n,
                             (int64_t)h.tl64.gemm.size(), h.mf.n_fronts, h.mf.n_levels, mx_f};
            (void)h.tl64.pairs.size();
            std::memcpy(sizes, v, sizeof(v));
        }
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_debug_mortar_blocks(const hplmm_system *sys, const hplmm_partition *part,
                                                  const hplmm_mortar *mortar, double *out, int64_t cap,
                                                  int64_t *needed) {
    return guarded([&]() -> hplmm_status {
        if (!sys || !part || !mortar) fail(HPLMM_E_ARG, "NULL argument");
        if (cap < 0 || (cap > 0 && !out)) fail(HPLMM_E_ARG, "bad output buffer");
        Handle h;
        hplmm_options o{64, 0};
        build_plan(h, *sys, *part, *mortar, o, nullptr, true);
        if (needed) *needed = (int64_t)h.h_H.size();
        if (out) std::memcpy(out, h.h_H.data(), sizeof(double) * (size_t)std::min<int64_t>(cap, (int64_t)h.h_H.size()));
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_setup(hplmm_handle *hh, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!hh) fail(HPLMM_E_ARG, "NULL handle");
        hh->h.ready = false;
        numeric_setup(hh->h, as_stream(stream));
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_setup_surrogate(hplmm_handle *hh, hplmm_sg_net *net, double threshold,
                                              hplmm_sg_stats *stats, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!hh || !net) fail(HPLMM_E_ARG, "NULL argument");
        if (!(threshold >= 0.0)) fail(HPLMM_E_ARG, "threshold must be >= 0");
        hh->h.ready = false;
        const SgSetup sg{net, threshold, stats};
        numeric_setup(hh->h, as_stream(stream), 3, &sg);
        return HPLMM_OK;
    });
}

// ---- autotuning of the solve-phase GEMV launches ------------------------------
// The smoother / basis GEMV launches of M^-1 in a fixed order (the index of
// their tuning records), with the vectors they read and write.
struct SetLaunch {
    Range *r;
    bool low;
    const double *x;
    double *y;
};
static std::vector<SetLaunch> set_launches(Handle &h) {
    const bool low = h.smoother_precision != 64;
    if (h.smoother_form == HPLMM_SMOOTHER_INVERSE)
        return {{&h.gset.gemv_S, false, h.gx, h.gy},
                {&h.cset.gemv_S, false, h.cx, h.cy},
                {&h.gemv_XT, false, h.gx, h.gc_t},
                {&h.gemv_X, false, h.gc_u, h.gy}};
    return {{&h.gset.gemv_W, low, h.gx, h.gt},   {&h.gset.gemv_Wt, low, h.gt, h.gy},
            {&h.cset.gemv_W, low, h.cx, h.ct},   {&h.cset.gemv_Wt, low, h.ct, h.cy},
            {&h.gemv_XT, false, h.gx, h.gc_t},   {&h.gemv_X, false, h.gc_u, h.gy}};
}

// Mean duration of fn in us: one warm-up call, then the best of three
// intervals of reps back-to-back calls timed with events on s.
template <class F>
static double time_us(hipStream_t s, int32_t reps, hipEvent_t e0, hipEvent_t e1, F fn) {
    fn();
    float best = 0.f;
    for (int trial = 0; trial < 3; ++trial) {
        hip_check(hipEventRecord(e0, s), "event");
        for (int32_t r = 0; r < reps; ++r) fn();
        hip_check(hipEventRecord(e1, s), "event");
        hip_check(hipEventSynchronize(e1), "sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        if (trial == 0 || ms < best) best = ms;
    }
    return 1e3 * best / reps;
}

// Median time (us) of fn run alone after the caches are overwritten by a
// triad over `flush` (three arrays of flush_n doubles, larger than L2 and
// the last-level cache together): a coarse-sweep launch reads its operators
// once per application, so it is timed as the sweep meets them.
template <class F>
static double time_cold_us(hipStream_t s, int32_t reps, hipEvent_t e0, hipEvent_t e1, double *flush, int64_t flush_n,
                           F fn) {
    fn();
    std::vector<float> t;
    for (int32_t r = 0; r < reps; ++r) {
        launch_triad(flush, flush + flush_n, flush + 2 * flush_n, 1.0, flush_n, s);
        hip_check(hipEventRecord(e0, s), "event");
        fn();
        hip_check(hipEventRecord(e1, s), "event");
        hip_check(hipEventSynchronize(e1), "sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    return 1e3 * t[t.size() / 2];
}

// Put the chosen shapes in place: coarse levels from their variant lists,
// smoother / basis launches by their waves.
static void apply_tuning(Handle &h, const std::vector<TuneRecord> &log) {
    CoarseMF &mf = h.mf;
    const auto sets = set_launches(h);
    for (const TuneRecord &t : log) {
        if (t.kind == 0 || t.kind == 1) {
            if (t.index < 0 || t.index >= mf.n_levels) fail(HPLMM_E_ARG, "tuning: level out of range");
            const GemvShapes &g = (t.kind == 0 ? mf.fwd_shapes : mf.bwd_shapes)[(size_t)t.index];
            if (t.variant < 0 || t.variant >= (int32_t)g.var.size()) fail(HPLMM_E_ARG, "tuning: variant out of range");
            Range r = g.var[(size_t)t.variant];
            r.waves = t.waves;
            (t.kind == 0 ? mf.fwd : mf.bwd)[(size_t)t.index] = r;
        } else if (t.kind == 2) {
            if (t.index < 0 || t.index >= (int32_t)sets.size()) fail(HPLMM_E_ARG, "tuning: launch out of range");
            sets[(size_t)t.index].r->waves = t.waves;
        } else {
            fail(HPLMM_E_ARG, "tuning: unknown launch kind");
        }
        if (t.waves != 4 && t.waves != 16) fail(HPLMM_E_ARG, "tuning: waves must be 4 or 16");
    }
}

static void default_tuning(Handle &h) {
    CoarseMF &mf = h.mf;
    for (int32_t l = 0; l < mf.n_levels; ++l) {
        mf.fwd[(size_t)l] = mf.fwd_shapes[(size_t)l].var[0];
        mf.bwd[(size_t)l] = mf.bwd_shapes[(size_t)l].var[0];
    }
    for (auto &sl : set_launches(h)) sl.r->waves = 4;
    h.tune_log.clear();
}

static void autotune(Handle &h, int32_t reps, hipStream_t s) {
    CoarseMF &mf = h.mf;
    default_tuning(h);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hip_check(hipEventCreate(&e0), "event");
    const hipError_t ec = hipEventCreate(&e1);
    if (ec != hipSuccess) {
        (void)hipEventDestroy(e0);
        hip_check(ec, "event");
    }
    std::vector<TuneRecord> log;
    try {
        // the sweeps run on zeroed front vectors: their in-place updates stay
        // zero.  Each shape is timed cold (see time_cold_us): repeated alone,
        // a level's operators stay cached, which flatters long unsplit rows.
        if (mf.n_fronts) zero(mf.V, sizeof(double) * 3 * (size_t)mf.vec_len, s);
        constexpr int64_t flush_n = (int64_t)1 << 24;   // 3 x 128 MiB
        double *flush = nullptr;
        if (mf.n_fronts) {
            hip_check(hipMalloc(&flush, sizeof(double) * 3 * flush_n), "hipMalloc");
            zero(flush, sizeof(double) * 3 * flush_n, s);
        }
        struct Free {
            double *p;
            ~Free() {
                if (p) (void)hipFree(p);
            }
        } free_flush{flush};
        const int32_t creps = std::max<int32_t>(3, reps / 2);
        for (int32_t kind = 0; kind < 2; ++kind)
            for (int32_t l = 0; l < mf.n_levels; ++l) {
                const GemvShapes &g = (kind == 0 ? mf.fwd_shapes : mf.bwd_shapes)[(size_t)l];
                if (g.var.empty() || g.var[0].count == 0) continue;
                TuneRecord best{kind, l, 0, g.target[0], 4, 0.0, 0.0};
                for (int32_t v = 0; v < (int32_t)g.var.size(); ++v)
                    for (int32_t w : {4, 16}) {
                        Range r = g.var[(size_t)v];
                        r.waves = w;
                        const double t = time_cold_us(s, creps, e0, e1, flush, flush_n, [&] { gemv_front(h, r, s); });
                        if (v == 0 && w == 4) best.t_default_us = best.t_best_us = t;
                        else if (t < best.t_best_us) {
                            best.variant = v;
                            best.target = g.target[(size_t)v];
                            best.waves = w;
                            best.t_best_us = t;
                        }
                    }
                log.push_back(best);
            }
        const auto sets = set_launches(h);
        for (int32_t i = 0; i < (int32_t)sets.size(); ++i) {
            const SetLaunch &sl = sets[(size_t)i];
            if (sl.r->count == 0) continue;
            TuneRecord best{2, i, 0, 0, 4, 0.0, 0.0};
            for (int32_t w : {4, 16}) {
                Range r = *sl.r;
                r.waves = w;
                const double t = time_us(s, reps, e0, e1, [&] { launch_set(h, r, sl.low, sl.x, sl.y, s); });
                if (w == 4) best.t_default_us = best.t_best_us = t;
                else if (t < best.t_best_us) {
                    best.waves = w;
                    best.t_best_us = t;
                }
            }
            log.push_back(best);
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    apply_tuning(h, log);
    h.tune_log = log;
}

extern "C" hplmm_status hplmm_autotune(hplmm_handle *hh, int32_t reps, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!hh) fail(HPLMM_E_ARG, "NULL handle");
        Handle &h = hh->h;
        if (!h.ready) fail(HPLMM_E_STATE, "hplmm_setup has not completed");
        if (reps < 1 || reps > 1000) fail(HPLMM_E_ARG, "reps must be 1..1000");
        const int32_t mask = h.prof.mask;
        h.prof.mask = 0;
        h.drop_graphs();   // captured steps hold the old launch shapes
        try {
            autotune(h, reps, (hipStream_t)stream);
        } catch (...) {
            h.prof.mask = mask;
            default_tuning(h);
            throw;
        }
        h.prof.mask = mask;
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_set_tuning(hplmm_handle *hh, const int32_t *rec, int64_t n) {
    return guarded([&]() -> hplmm_status {
        if (!hh) fail(HPLMM_E_ARG, "NULL handle");
        Handle &h = hh->h;
        if (n < 0 || (n > 0 && !rec)) fail(HPLMM_E_ARG, "bad tuning records");
        hip_check(hipDeviceSynchronize(), "sync");
        h.drop_graphs();
        default_tuning(h);
        std::vector<TuneRecord> log;
        for (int64_t i = 0; i < n; ++i) {
            const int32_t *q = rec + 4 * i;
            TuneRecord t{q[0], q[1], q[2], 0, q[3], 0.0, 0.0};
            if ((t.kind == 0 || t.kind == 1) && t.index >= 0 && t.index < h.mf.n_levels) {
                const GemvShapes &g = (t.kind == 0 ? h.mf.fwd_shapes : h.mf.bwd_shapes)[(size_t)t.index];
                if (t.variant >= 0 && t.variant < (int32_t)g.target.size()) t.target = g.target[(size_t)t.variant];
            }
            log.push_back(t);
        }
        try {
            apply_tuning(h, log);
        } catch (...) {
            default_tuning(h);
            throw;
        }
        h.tune_log = log;
        return HPLMM_OK;
    });
}

// ---- matrix-free fine operator --------------------------------------------------
extern "C" hplmm_status hplmm_set_voxel_operator(hplmm_handle *hh, int32_t nx, int32_t ny, int32_t nz,
                                                 const uint8_t *solid, const double *E, double nu, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!hh) fail(HPLMM_E_ARG, "NULL handle");
        Handle &h = hh->h;
        if (h.n_fixed > 0 && (nx | ny | nz) != 0)
            fail(HPLMM_E_ARG, "the matrix-free operator knows the clamped plane only, not constrained dofs");
        const hipStream_t s = (hipStream_t)stream;
        hip_check(hipStreamSynchronize(s), "sync");
        h.drop_graphs();   // captured steps hold the old operator
        if (h.spmv_bytes_assembled < 0.0) {
            h.spmv_bytes_assembled = h.spmv_bytes;
            h.apply_bytes_assembled = h.apply_bytes;
        }
        if (nx == 0 && ny == 0 && nz == 0) {
            h.vop_on = false;
            h.spmv_bytes = h.spmv_bytes_assembled;
            h.apply_bytes = h.apply_bytes_assembled;
            return HPLMM_OK;
        }
        if (nx < 1 || ny < 1 || nz < 1) fail(HPLMM_E_ARG, "grid dimensions must be positive (all zero: assembled operator)");
        const int64_t nvox = (int64_t)nx * ny * nz;
        if (nvox > ((int64_t)1 << 31)) fail(HPLMM_E_ARG, "more than 2^31 voxels");
        if (!solid || !E) fail(HPLMM_E_ARG, "NULL array");
        if (!(nu > -1.0 && nu < 0.5)) fail(HPLMM_E_ARG, "nu must lie in (-1, 0.5)");
        for (int64_t q = 0; q < nvox; ++q)
            if (solid[q] && !(std::isfinite(E[q]) && E[q] >= 0.0)) fail(HPLMM_E_ARG, "E must be finite and >= 0 on solid voxels");
        // lattice point -> free node, from the planned node coordinates
        const int64_t NX = nx + 1, NY = ny + 1, NZ = nz + 1;
        std::vector<int32_t> lat((size_t)(NX * NY * NZ), -1);
        for (int64_t v = 0; v < h.n_nodes; ++v) {
            const int32_t i = h.sg_xyz[(size_t)(3 * v)], j = h.sg_xyz[(size_t)(3 * v + 1)], k = h.sg_xyz[(size_t)(3 * v + 2)];
            if (i < 0 || j < 0 || k < 0 || i > nx || j > ny || k > nz) fail(HPLMM_E_ARG, "a node lies outside the grid");
            int32_t &slot = lat[(size_t)(i + NX * (j + NY * (int64_t)k))];
            if (slot >= 0) fail(HPLMM_E_ARG, "two nodes share a lattice point");
            slot = (int32_t)v;
        }
        double K[24][24];
        q1_element_stiffness(nu, K);
        const std::vector<uint8_t> vs(solid, solid + nvox);
        const std::vector<double> ve(E, E + nvox), vk(&K[0][0], &K[0][0] + 24 * 24);
        // the padded copies the matrix-free operator reads (halo of void
        // voxels and of lattice points without a node)
        const int64_t PX = nx + 2, PY = ny + 2, PZ = nz + 2, QX = nx + 3, QY = ny + 3, QZ = nz + 3;
        std::vector<double> ep((size_t)(PX * PY * PZ), 0.0);
        for (int64_t ez = 0; ez < nz; ++ez)
            for (int64_t ey = 0; ey < ny; ++ey)
                for (int64_t ex = 0; ex < nx; ++ex) {
                    const int64_t q = ex + nx * (ey + ny * ez);
                    if (solid[q]) ep[(size_t)((ex + 1) + PX * ((ey + 1) + PY * (ez + 1)))] = E[q];
                }
        std::vector<int32_t> lp((size_t)(QX * QY * QZ), -1);
        for (int64_t c = 0; c < NZ; ++c)
            for (int64_t b = 0; b < NY; ++b)
                for (int64_t a = 0; a < NX; ++a)
                    lp[(size_t)((a + 1) + QX * ((b + 1) + QY * (c + 1)))] = lat[(size_t)(a + NX * (b + NY * c))];
        VoxelGrid g{nx, ny, nz, h.upload(vs, s), h.upload(ve, s), nu, h.upload(lat, s), h.n_nodes,
                    h.upload(ep, s), h.upload(lp, s)};
        const int32_t *xyz = h.upload(h.sg_xyz, s);
        const double *Kd = h.upload(vk, s);
        // the two operators on one seeded vector must agree to rounding
        const int64_t N = h.N;
        std::vector<double> xr((size_t)N), y1((size_t)N), y2((size_t)N);
        uint64_t st = 0x9e3779b97f4a7c15ull;
        for (auto &v : xr) {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            v = (double)(st >> 11) * (2.0 / 9007199254740992.0) - 1.0;
        }
        double *dx = h.upload(xr, s), *dy1 = h.dalloc<double>(N), *dy2 = h.dalloc<double>(N);
        launch_spmv(h.sell, dx, nullptr, dy1, s);
        launch_spmv_voxel(g, xyz, Kd, dx, nullptr, dy2, s);
        hip_check(hipGetLastError(), "kernel launch");
        hip_check(hipMemcpyAsync(y1.data(), dy1, sizeof(double) * (size_t)N, hipMemcpyDeviceToHost, s), "copy");
        hip_check(hipMemcpyAsync(y2.data(), dy2, sizeof(double) * (size_t)N, hipMemcpyDeviceToHost, s), "copy");
        hip_check(hipStreamSynchronize(s), "sync");
        double mx = 0.0, md = 0.0;
        for (int64_t q = 0; q < N; ++q) {
            mx = std::max(mx, std::fabs(y1[(size_t)q]));
            md = std::max(md, std::fabs(y1[(size_t)q] - y2[(size_t)q]));
        }
        if (!(md <= 1e-12 * mx))
            fail(HPLMM_E_ARG, "the voxel operator differs from the assembled matrix (max |difference| " +
                                  std::to_string(md) + " against max |A x| " + std::to_string(mx) + ")");
        h.vop = g;
        h.vop_xyz = xyz;
        h.vop_K = Kd;
        h.vop_on = true;
        // algorithmic bytes: x read and y written per node, the voxel grid and the lattice map
        const double mf = (double)h.n_nodes * 48.0 + (double)nvox * 9.0 + (double)lat.size() * 4.0;
        h.spmv_bytes = mf;
        h.apply_bytes = h.apply_bytes_assembled - 2.0 * h.spmv_bytes_assembled + 2.0 * mf;
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_use_graphs(hplmm_handle *hh, int32_t on) {
    return guarded([&]() -> hplmm_status {
        if (!hh) fail(HPLMM_E_ARG, "NULL handle");
        hh->h.use_graphs = on != 0;
        if (!on) hh->h.drop_graphs();
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_apply(hplmm_handle *hh, int32_t which, const double *r, double *z, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!hh || !r || !z) fail(HPLMM_E_ARG, "NULL argument");
        if (r == z) fail(HPLMM_E_ARG, "r and z must not alias");
        if (!hh->h.ready) fail(HPLMM_E_STATE, "hplmm_setup has not completed");
        apply_op(hh->h, which, r, z, as_stream(stream));
        hip_check(hipGetLastError(), "kernel launch");
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_spmv(hplmm_handle *hh, const double *x, double *y, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!hh || !x || !y) fail(HPLMM_E_ARG, "NULL argument");
        if (x == y) fail(HPLMM_E_ARG, "x and y must not alias");
        spmv(hh->h, x, nullptr, y, as_stream(stream));
        hip_check(hipGetLastError(), "kernel launch");
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_solve(hplmm_handle *hh, const double *b, double *x, double rtol, int32_t restart,
                                    int32_t maxit, int32_t fixed_iters, hplmm_solve_info *info, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!hh || !b || !x) fail(HPLMM_E_ARG, "NULL argument");
        if (b == x) fail(HPLMM_E_ARG, "b and x must not alias");
        if (!hh->h.ready) fail(HPLMM_E_STATE, "hplmm_setup has not completed");
        if (restart < 1 || restart > 120 || maxit < 0) fail(HPLMM_E_ARG, "restart must be in [1, 120], maxit >= 0");
        const auto t0 = std::chrono::steady_clock::now();
        const hplmm_status st = gmres(hh->h, b, x, rtol, restart, maxit, fixed_iters, info, as_stream(stream));
        const auto t1 = std::chrono::steady_clock::now();
        if (info) {
            info->t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
            info->t_ml_ms = hh->h.t_ml_ms;
            info->t_mg_ms = hh->h.t_mg_ms;
        }
        return st;
    });
}

extern "C" hplmm_status hplmm_query(hplmm_handle *hh, int32_t what, void *out, int64_t cap, int64_t *needed) {
    return guarded([&]() -> hplmm_status {
        if (!hh) fail(HPLMM_E_ARG, "NULL handle");
        Handle &h = hh->h;
        std::vector<char> buf;
        auto put = [&](const void *p, size_t n) { buf.insert(buf.end(), (const char *)p, (const char *)p + n); };
        switch (what) {
            case 0: {
                int64_t mx_g = 0, mx_c = 0;
                for (auto v : h.gset.n) mx_g = std::max(mx_g, v);
                for (auto v : h.cset.n) mx_c = std::max(mx_c, v);
                int64_t mx_f = 0;
                for (int32_t t = 0; t < h.mf.n_fronts; ++t) mx_f = std::max(mx_f, h.mf.d[(size_t)t] + h.mf.u[(size_t)t]);
                int64_t v[16] = {h.n_nodes, h.nnzb, h.n_grains, h.n_ifaces, h.n_contacts, h.n_mortar, h.n_corr,
                                 h.n_coarse, (int64_t)h.gset.n.size(), mx_g, mx_c, h.sell.n_slices,
                                 h.sell_padded_blocks, h.mf.n_fronts, h.mf.n_levels, mx_f};
                put(v, sizeof(v));
                break;
            }
            case 1: put(h.h_mortar_idx.data(), sizeof(int32_t) * h.h_mortar_idx.size()); break;
            case 2: put(h.h_H.data(), sizeof(double) * h.h_H.size()); break;
            case 3: put(h.h_corr_grains.data(), sizeof(int32_t) * h.h_corr_grains.size()); break;
            case 4: {
                if (!h.ready) fail(HPLMM_E_STATE, "hplmm_setup has not completed");
                const int64_t nc = h.n_coarse;
                if (nc > 8000) fail(HPLMM_E_ARG, "coarse matrix too large to return densely");
                std::vector<double> vals((size_t)h.n_pair_vals), cd((size_t)h.n_corr);
                if (h.n_pair_vals)
                    hip_check(hipMemcpy(vals.data(), h.pair_vals, sizeof(double) * vals.size(), hipMemcpyDeviceToHost), "copy");
                if (h.n_corr)
                    hip_check(hipMemcpy(cd.data(), h.corr_d, sizeof(double) * cd.size(), hipMemcpyDeviceToHost), "copy");
                std::vector<int32_t> nu((size_t)h.n_ifaces);
                std::vector<int64_t> mo((size_t)h.n_ifaces);
                hip_check(hipMemcpy(nu.data(), h.cm.iface_nu, sizeof(int32_t) * nu.size(), hipMemcpyDeviceToHost), "copy");
                hip_check(hipMemcpy(mo.data(), h.cm.iface_moff, sizeof(int64_t) * mo.size(), hipMemcpyDeviceToHost), "copy");
                std::vector<double> S((size_t)(nc * nc), 0.0);
                for (const auto &pr : h.h_pairs) {
                    const int n1 = 3 * nu[(size_t)pr.c], n2 = 3 * nu[(size_t)pr.c2];
                    for (int i = 0; i < n1; ++i)
                        for (int j = 0; j < n2; ++j) {
                            const int64_t p = mo[(size_t)pr.c] + i, q = mo[(size_t)pr.c2] + j;
                            const double v = vals[(size_t)(pr.v_off + (int64_t)i * n2 + j)];
                            if (pr.c == pr.c2 && i < j) continue;
                            S[(size_t)(p * nc + q)] = v;
                            S[(size_t)(q * nc + p)] = v;
                        }
                }
                for (int64_t j = 0; j < h.n_corr; ++j) S[(size_t)((h.n_mortar + j) * nc + h.n_mortar + j)] = cd[(size_t)j];
                put(S.data(), sizeof(double) * S.size());
                break;
            }
            case 5: put(h.t_setup_ms, sizeof(h.t_setup_ms)); break;
            case 7: {
                hip_check(hipDeviceSynchronize(), "sync");
                std::vector<double> acc(3 * PC_COUNT, 0.0);
                for (const auto &rc : h.prof.recs) {
                    float ms = 0.f;
                    hip_check(hipEventElapsedTime(&ms, h.prof.pool[rc.ev], h.prof.pool[rc.ev + 1]), "elapsed");
                    acc[(size_t)(3 * rc.cls)] += 1.0;
                    acc[(size_t)(3 * rc.cls + 1)] += ms;
                    acc[(size_t)(3 * rc.cls + 2)] += rc.units;
                }
                put(acc.data(), sizeof(double) * acc.size());
                break;
            }
            case 8: {
                const double v[2] = {h.apply_bytes, h.spmv_bytes};
                put(v, sizeof(v));
                break;
            }
            case 6: put(&h.dev_bytes, sizeof(int64_t)); break;
            case 9: {
                std::vector<double> v;
                for (int32_t l = 0; l < h.mf.n_levels; ++l) {
                    int64_t nf = 0;
                    for (int32_t t = 0; t < h.mf.n_fronts; ++t) nf += h.mf.level[(size_t)t] == l;
                    const Range &f = h.mf.fwd[(size_t)l], &b = h.mf.bwd[(size_t)l];
                    for (double x : {(double)nf, (double)f.count, f.bytes, (double)b.count, b.bytes}) v.push_back(x);
                }
                put(v.data(), sizeof(double) * v.size());
                break;
            }
            case 10: {
                std::vector<double> v;
                for (const TuneRecord &t : h.tune_log)
                    for (double x : {(double)t.kind, (double)t.index, (double)t.variant, (double)t.target,
                                     (double)t.waves, t.t_default_us, t.t_best_us})
                        v.push_back(x);
                put(v.data(), sizeof(double) * v.size());
                break;
            }
            case 11: put(&h.smoother_form, sizeof(int32_t)); break;
            case 13: {
                double v[13];
                std::memcpy(v, h.method_setup_flops, sizeof(h.method_setup_flops));
                std::memcpy(v + 4, h.issued_setup_flops, sizeof(h.issued_setup_flops));
                std::memcpy(v + 8, h.method_apply_bytes, sizeof(h.method_apply_bytes));
                put(v, sizeof(v));
                break;
            }
            case 12: {
                const int64_t v[1] = {h.gemv_part_len};
                put(v, sizeof(v));
                break;
            }
            default: fail(HPLMM_E_ARG, "unknown query");
        }
        if (needed) *needed = (int64_t)buf.size();
        if (out && cap > 0) std::memcpy(out, buf.data(), (size_t)std::min<int64_t>(cap, (int64_t)buf.size()));
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_profile(hplmm_handle *hh, int32_t mask) {
    return guarded([&]() -> hplmm_status {
        if (!hh) fail(HPLMM_E_ARG, "NULL handle");
        hip_check(hipDeviceSynchronize(), "sync");
        hh->h.prof.mask = mask;
        hh->h.prof.recs.clear();
        hh->h.prof.used = 0;
        return HPLMM_OK;
    });
}

extern "C" void hplmm_destroy(hplmm_handle *hh) {
    if (!hh) return;
    (void)hipDeviceSynchronize();
    delete hh;
}

// ---- test hooks ---------------------------------------------------------------------
extern "C" hplmm_status hplmm_debug_tile_gemm(int32_t precision, const void *A, const void *B, int32_t npairs,
                                              const void *Pm, void *Cm, int32_t flags, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (precision == 16) {
            // bfloat16 operands, FP32 C: contraction flags only
            if (!A || !B || !Cm || npairs < 1) fail(HPLMM_E_ARG, "bad arguments");
            if (flags & ~(GF_TRANS_A | GF_TRANS_B | GF_ACCUM | GF_NEGATE)) fail(HPLMM_E_ARG, "flag not available");
            hipStream_t s = as_stream(stream);
            uint16_t *in = nullptr;
            float *out = nullptr;
            GemmTask *dt = nullptr;
            GemmPair *dp = nullptr;
            hip_check(hipMalloc(&in, sizeof(uint16_t) * TE * 2 * (size_t)npairs), "hipMalloc");
            hip_check(hipMalloc(&out, sizeof(float) * TE), "hipMalloc");
            hip_check(hipMemcpyAsync(in, A, sizeof(uint16_t) * TE * npairs, hipMemcpyDeviceToDevice, s), "copy");
            hip_check(hipMemcpyAsync(in + (size_t)TE * npairs, B, sizeof(uint16_t) * TE * npairs,
                                     hipMemcpyDeviceToDevice, s), "copy");
            hip_check(hipMemcpyAsync(out, Cm, sizeof(float) * TE, hipMemcpyDeviceToDevice, s), "copy");
            std::vector<GemmPair> pr;
            for (int32_t p = 0; p < npairs; ++p) pr.push_back({(int64_t)p * TE, (int64_t)(npairs + p) * TE});
            GemmTask t{0, -1, 0, npairs, flags, 0};
            hip_check(hipMalloc(&dt, sizeof(t)), "hipMalloc");
            hip_check(hipMalloc(&dp, sizeof(GemmPair) * pr.size()), "hipMalloc");
            hip_check(hipMemcpyAsync(dt, &t, sizeof(t), hipMemcpyHostToDevice, s), "copy");
            hip_check(hipMemcpyAsync(dp, pr.data(), sizeof(GemmPair) * pr.size(), hipMemcpyHostToDevice, s), "copy");
            launch_tile_gemm_bf16(in, out, dt, dp, 1, s);
            hip_check(hipMemcpyAsync(Cm, out, sizeof(float) * TE, hipMemcpyDeviceToDevice, s), "copy");
            hip_check(hipStreamSynchronize(s), "sync");
            (void)hipFree(in);
            (void)hipFree(out);
            (void)hipFree(dt);
            (void)hipFree(dp);
            return HPLMM_OK;
        }
        if (!A || !B || !Cm || npairs < 0 || (precision != 64 && precision != 32)) fail(HPLMM_E_ARG, "bad arguments");
        if (flags & ~(GF_TRANS_A | GF_TRANS_B | GF_ACCUM | GF_NEGATE | GF_POST | GF_POST_RIGHT))
            fail(HPLMM_E_ARG, "unknown flag");
        if ((flags & GF_POST) && (flags & GF_POST_RIGHT)) fail(HPLMM_E_ARG, "GF_POST and GF_POST_RIGHT exclude each other");
        if ((flags & (GF_POST | GF_POST_RIGHT)) && !Pm) fail(HPLMM_E_ARG, "P needed");
        if (npairs == 0 && !(flags & GF_POST_RIGHT)) fail(HPLMM_E_ARG, "no pairs");
        hipStream_t s = as_stream(stream);
        const size_t es = precision == 64 ? 8 : 4;
        // gather everything into one scratch arena: [A tiles][B tiles][P][C]
        const int64_t n_el = (int64_t)(2 * npairs + 2) * TE;
        void *ar = nullptr;
        hip_check(hipMalloc(&ar, es * (size_t)n_el), "hipMalloc");
        char *base = (char *)ar;
        hip_check(hipMemcpyAsync(base, A, es * TE * npairs, hipMemcpyDeviceToDevice, s), "copy");
        hip_check(hipMemcpyAsync(base + es * TE * npairs, B, es * TE * npairs, hipMemcpyDeviceToDevice, s), "copy");
        if (Pm) hip_check(hipMemcpyAsync(base + es * TE * 2 * npairs, Pm, es * TE, hipMemcpyDeviceToDevice, s), "copy");
        hip_check(hipMemcpyAsync(base + es * TE * (2 * npairs + 1), Cm, es * TE, hipMemcpyDeviceToDevice, s), "copy");
        std::vector<GemmPair> pr;
        for (int32_t p = 0; p < npairs; ++p) pr.push_back({(int64_t)p * TE, (int64_t)(npairs + p) * TE});
        GemmTask t{(int64_t)(2 * npairs + 1) * TE, (int64_t)(2 * npairs) * TE, 0, npairs, flags, 0};
        GemmTask *dt = nullptr;
        GemmPair *dp = nullptr;
        hip_check(hipMalloc(&dt, sizeof(t)), "hipMalloc");
        hip_check(hipMalloc(&dp, sizeof(GemmPair) * std::max<size_t>(1, pr.size())), "hipMalloc");
        hip_check(hipMemcpyAsync(dt, &t, sizeof(t), hipMemcpyHostToDevice, s), "copy");
        if (!pr.empty())
            hip_check(hipMemcpyAsync(dp, pr.data(), sizeof(GemmPair) * pr.size(), hipMemcpyHostToDevice, s), "copy");
        if (precision == 64)
            launch_tile_gemm<double>((double *)ar, dt, dp, 1, s);
        else
            launch_tile_gemm<float>((float *)ar, dt, dp, 1, s);
        hip_check(hipMemcpyAsync(Cm, base + es * TE * (2 * npairs + 1), es * TE, hipMemcpyDeviceToDevice, s), "copy");
        hip_check(hipStreamSynchronize(s), "sync");
        (void)hipFree(ar);
        (void)hipFree(dt);
        (void)hipFree(dp);
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_debug_diag(int32_t precision, void *A, const void *P, void *W, void *Wt, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!A || !W || !Wt || (precision != 64 && precision != 32)) fail(HPLMM_E_ARG, "bad arguments");
        hipStream_t s = as_stream(stream);
        const size_t es = precision == 64 ? 8 : 4;
        void *ar = nullptr;
        hip_check(hipMalloc(&ar, es * 4 * TE), "hipMalloc");
        char *base = (char *)ar;
        hip_check(hipMemcpyAsync(base, A, es * TE, hipMemcpyDeviceToDevice, s), "copy");
        if (P) hip_check(hipMemcpyAsync(base + es * 3 * TE, P, es * TE, hipMemcpyDeviceToDevice, s), "copy");
        DiagTask t{0, TE, 2 * TE, 7, 0, P ? 3 * TE : -1};
        DiagTask *dt = nullptr;
        int32_t *flag = nullptr;
        hip_check(hipMalloc(&dt, sizeof(t)), "hipMalloc");
        hip_check(hipMalloc(&flag, 8), "hipMalloc");
        const int32_t f0[2] = {0, 0x7fffffff};
        hip_check(hipMemcpyAsync(flag, f0, 8, hipMemcpyHostToDevice, s), "copy");
        hip_check(hipMemcpyAsync(dt, &t, sizeof(t), hipMemcpyHostToDevice, s), "copy");
        if (precision == 64)
            launch_diag<double>((double *)ar, (double *)ar, (double *)ar, dt, 1, flag, s);
        else
            launch_diag<float>((float *)ar, (float *)ar, (float *)ar, dt, 1, flag, s);
        hip_check(hipMemcpyAsync(A, base, es * TE, hipMemcpyDeviceToDevice, s), "copy");
        hip_check(hipMemcpyAsync(W, base + es * TE, es * TE, hipMemcpyDeviceToDevice, s), "copy");
        hip_check(hipMemcpyAsync(Wt, base + 2 * es * TE, es * TE, hipMemcpyDeviceToDevice, s), "copy");
        int32_t fl[2];
        hip_check(hipMemcpyAsync(fl, flag, 8, hipMemcpyDeviceToHost, s), "copy");
        hip_check(hipStreamSynchronize(s), "sync");
        (void)hipFree(ar);
        (void)hipFree(dt);
        (void)hipFree(flag);
        if (fl[0]) fail(HPLMM_E_NOT_SPD, "non-positive pivot");
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_stream_triad(double *a, const double *b, const double *c, double scalar, int64_t n,
                                           void *stream) {
    return guarded([&]() -> hplmm_status {
        if (n < 0 || (n > 0 && (!a || !b || !c))) fail(HPLMM_E_ARG, "bad arguments");
        if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15) fail(HPLMM_E_ARG, "arrays must be 16-byte aligned");
        launch_triad(a, b, c, scalar, n, as_stream(stream));
        hip_check(hipGetLastError(), "triad launch");
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_debug_setup_stage(hplmm_handle *hh, int32_t stage, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!hh) fail(HPLMM_E_ARG, "NULL handle");
        hh->h.ready = false;
        numeric_setup(hh->h, as_stream(stream), stage);
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_debug_read_arena(hplmm_handle *hh, int32_t arena, int64_t off, int64_t count,
                                               void *out) {
    return guarded([&]() -> hplmm_status {
        if (!hh || !out || off < 0 || count < 0) fail(HPLMM_E_ARG, "bad arguments");
        Handle &h = hh->h;
        const void *base = arena == 0 ? (const void *)h.ar64 : arena == 1 ? (const void *)h.ar32 : (const void *)h.arbf;
        const int64_t n = arena == 0 ? h.ar64_n : arena == 1 ? h.ar32_n : h.arbf_n;
        const size_t es = arena == 0 ? 8 : arena == 1 ? 4 : 2;
        if (off + count > n) fail(HPLMM_E_ARG, "range outside the arena");
        hip_check(hipDeviceSynchronize(), "sync");
        hip_check(hipMemcpy(out, (const char *)base + es * off, es * count, hipMemcpyDeviceToHost), "copy");
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_debug_grain_layout(hplmm_handle *hh, int64_t *out, int64_t cap) {
    return guarded([&]() -> hplmm_status {
        if (!hh || !out) fail(HPLMM_E_ARG, "bad arguments");
        Handle &h = hh->h;
        const int64_t nm = (int64_t)h.gset.n.size();
        if (cap < 11 * nm) fail(HPLMM_E_ARG, "buffer too small");
        for (int64_t m = 0; m < nm; ++m) {
            int64_t *o = out + 11 * m;
            o[0] = h.gm_grain[(size_t)m];
            o[1] = h.gset.n[(size_t)m];
            o[2] = h.gset.nt[(size_t)m];
            o[3] = h.gm_ncol[(size_t)m];
            o[4] = h.gm_ntc[(size_t)m];
            o[5] = h.gset.a_base + h.gset.rel[(size_t)m];
            o[6] = h.gset.w_base + h.gset.rel[(size_t)m];
            o[7] = h.gset.wt_diag ? -1 : h.gset.wt_base + h.gset.rel[(size_t)m];
            o[8] = h.gm_roff[(size_t)m];
            o[9] = h.gm_ytoff[(size_t)m];
            o[10] = h.gm_koff[(size_t)m];
        }
        return HPLMM_OK;
    });
}

extern "C" hplmm_status hplmm_debug_contact_layout(hplmm_handle *hh, int64_t *out, int64_t cap) {
    return guarded([&]() -> hplmm_status {
        if (!hh || !out) fail(HPLMM_E_ARG, "bad arguments");
        Handle &h = hh->h;
        const int64_t nm = (int64_t)h.cset.n.size();
        if (cap < 6 * nm) fail(HPLMM_E_ARG, "buffer too small");
        // the float32 factor form factors the contact grids in the float32 arena
        const bool f32 = h.smoother_precision != 64 && h.smoother_form == HPLMM_SMOOTHER_FACTORS;
        for (int64_t m = 0; m < nm; ++m) {
            int64_t *o = out + 6 * m;
            o[0] = h.cset.n[(size_t)m];
            o[1] = h.cset.nt[(size_t)m];
            o[2] = f32 ? 1 : 0;
            o[3] = h.cset.a_base + h.cset.rel[(size_t)m];
            o[4] = h.cset.w_base + h.cset.rel[(size_t)m];
            o[5] = h.cset.wt_diag ? -1 : h.cset.wt_base + h.cset.rel[(size_t)m];
        }
        return HPLMM_OK;
    });
}
