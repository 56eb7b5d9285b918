// Internal state of an hplmm_handle: sizes, device buffers, task lists.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "common.h"
#include "dense.h"
#include "sparse.h"
#include "post.h"
#include "surrogate.h"

namespace hplmm {

enum LaunchKind : int32_t { LK_DIAG = 0, LK_GEMM = 1, LK_TRANSPOSE = 2 };

struct Launch {
    int32_t kind;
    int64_t start;
    int64_t count;
    double flops = 0.0;   // algorithmic flops of the launch (2*64^3 per tile product)
    bool split = false;   // GEMM launches: some tasks split (a finishing pass follows)
};

// Kernel classes timed by the built-in profiler.
enum ProfClass : int32_t {
    PC_TILE_GEMM = 0,     // set-up tile contractions (units: flops)
    PC_DIAG = 1,          // diagonal-tile factorisations (units: tiles)
    PC_GEMV_SMOOTH = 2,   // smoother GEMVs, grain + contact (units: bytes)
    PC_GEMV_COARSE = 3,   // coarse solve GEMVs (units: bytes)
    PC_GEMV_BASIS = 4,    // restriction / prolongation GEMVs (units: bytes)
    PC_SPMV = 5,          // fine SpMV (units: bytes)
    PC_APPLY = 6,         // one whole preconditioner application (units: bytes)
    PC_SMOOTH_REDUCE = 7, // transposed-product sums of the symmetric smoother (units: bytes)
    PC_COUNT = 8
};

struct Profiler {
    int32_t mask = 0;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec {
        int32_t cls;
        size_t ev;
        double units;
    };
    std::vector<Rec> recs;
};

// Host-side task lists of one element type (uploaded once).
struct TaskLists {
    std::vector<GemmTask> gemm;
    std::vector<GemmPair> pairs;
    std::vector<DiagTask> diag;
    std::vector<CopyTask> copy;
    GemmTask *d_gemm = nullptr;
    GemmPair *d_pairs = nullptr;
    DiagTask *d_diag = nullptr;
    CopyTask *d_copy = nullptr;
    int64_t part_len = 0;        // split-task partial tiles (elements of the list's type)
    void *d_part = nullptr;
};

struct Range {
    int64_t start = 0, count = 0;
    double bytes = 0.0;   // algorithmic bytes read and written by the launch
    int32_t waves = 4;    // GEMV launches: wavefronts per work-group (4 or 16)
    bool sym = false;     // GEMV launches: symmetric-operator tasks (SymPair lists)
    bool split = false;   // GEMV launches: some rows split (a reduction launch follows)
};

// Launch shapes of one GEMV launch that the autotuner chooses from: the same
// rows emitted for several work-group targets (split rows, target 0 = as
// planned); var[0] is the default.
struct GemvShapes {
    std::vector<Range> var;
    std::vector<int32_t> target;
};

// One autotuned launch: kind 0/1 = coarse forward/backward sweep at level
// index, kind 2 = smoother / basis GEMV (index: grain W, grain W^T, contact
// W, contact W^T, X^T, X); the chosen variant, waves and timings (us).
struct TuneRecord {
    int32_t kind, index, variant, target, waves;
    double t_default_us, t_best_us;
};

// A batch of symmetric positive definite matrices stored as packed lower
// tiles; A (factored in place to L), W = L^-1 and Wt = L^-T share the same
// relative layout in three regions of one arena, and so does the inverse
// S = W^T W when the smoother applies it (s_base >= 0).
struct DenseSet {
    std::vector<int64_t> n, nt, rel;   // size, tiles per side, relative offset
    int64_t region = 0;                // elements per region
    int64_t a_base = 0, w_base = 0, wt_base = 0;   // absolute arena offsets
    int64_t s_base = -1;
    std::vector<Launch> factor_prog;   // potrf + trtri + transposes
    std::vector<Launch> w_prog;        // the rows of W = L^-1 when not fused into factor_prog
    std::vector<Launch> inverse_prog;  // S = W^T W (lower tiles)
    Range gemv_W, gemv_Wt;             // apply-time task ranges (factor form)
    Range gemv_S, red_S;               // apply-time task ranges (inverse form)
    int64_t vec_len = 0;               // local vector length (sum nt*64)
    std::vector<int64_t> voff;         // local vector offset per matrix
    int64_t low_w_base = 0, low_wt_base = 0;   // offsets in the reduced-precision arena
    int64_t low_s_base = 0;            // S as the smoother reads it (= s_base at FP64)
    std::vector<int64_t> nt_own;       // tiles factored per matrix (partial factorisation); empty = nt
    std::vector<int64_t> wrel;         // W / Wt relative offsets, only tri(nt_own) tiles each; empty = rel
    // Wt holds only the diagonal tiles W_kk^T (the inverse form, whose
    // products read W transposed instead): tile k of matrix m at wdrel[m] + k TE
    bool wt_diag = false;
    std::vector<int64_t> wdrel;
    // tile envelope: first[m][I] is the first tile column of row I of matrix
    // m that holds a nonzero; the Cholesky factor has none left of it.  Empty:
    // every matrix dense
    std::vector<std::vector<int32_t>> first;
};

// Multifrontal Cholesky of the coarse operator on a nested-dissection tree of
// interfaces.  Front t holds its own interfaces' dofs (padded to nt_d tiles)
// followed by its boundary dofs (padded to nt_u tiles) as packed lower tiles;
// its first nt_d tile columns are factored, leaving the update matrix in the
// boundary block.  Level 0 is the root.
struct CoarseMF {
    int32_t n_fronts = 0, n_levels = 0;
    std::vector<int32_t> parent, level, side;
    std::vector<int64_t> d, u, nt_d, nt_u, rel, wrel, ltrel, voff;   // wrel: W11 / W11^T, tri(nt_d) tiles each
    std::vector<std::vector<int32_t>> own, bnd;
    std::vector<int32_t> iface_front;
    std::vector<int64_t> iface_pos;           // position inside its owner front
    int64_t region = 0, w_region = 0, lt_region = 0, vec_len = 0;
    int64_t a_base = 0, w_base = 0, wt_base = 0, lt_base = 0, ng_base = 0;
    std::vector<std::vector<Launch>> factor_prog;   // per level
    std::vector<Range> ext_lvl;                     // per level: extend-add parent tiles
    std::vector<Range> vec_ext, bwd_copy;           // per level
    std::vector<Range> fwd, bwd;                    // per level: one GEMV launch each way (the chosen shape)
    std::vector<GemvShapes> fwd_shapes, bwd_shapes; // per level: the shapes the autotuner may pick
    std::vector<ExtendTile> ext;
    std::vector<int32_t> maps;
    std::vector<int32_t> inv;                       // parent position -> child boundary row or -1, per child
    std::vector<int64_t> inv_at;                    // per front: its inverse map in inv, -1 at the root
    std::vector<int64_t> va_dst, va_ptr, va_src, cp_dst, cp_src, init_map, out_dst, out_src;
    std::vector<int64_t> pad_ones;
    ExtendTile *d_ext = nullptr;
    int32_t *d_inv = nullptr;
    int64_t *d_va_dst = nullptr, *d_va_ptr = nullptr, *d_va_src = nullptr, *d_cp_dst = nullptr, *d_cp_src = nullptr;
    int64_t *d_init_map = nullptr, *d_out_dst = nullptr, *d_out_src = nullptr, *d_pad = nullptr;
    double *V = nullptr, *WV = nullptr, *YV = nullptr, *XV = nullptr;   // WV, YV, XV are views of V
    double flops = 0.0, factor_bytes = 0.0;
};

struct Handle {
    int device = 0;
    std::vector<void *> allocs;
    int64_t dev_bytes = 0;

    // sizes
    int64_t n_nodes = 0, N = 0, nnzb = 0;
    int32_t n_grains = 0, n_ifaces = 0, n_contacts = 0;
    int64_t n_mortar = 0, n_corr = 0, n_coarse = 0;
    int32_t smoother_precision = 64;
    int32_t mortar_kind = HPLMM_MORTAR_GAUSSIAN;
    int64_t coarse_leaf_dofs = 192;
    int64_t n_fixed = 0;   // constrained dofs (identity rows) of the planned system
    bool ready = false;

    // fine matrix
    FineCsr csr{};
    SellMatrix sell{};
    int64_t sell_padded_blocks = 0;
    double *d_b = nullptr;

    // interface and coarse maps
    CoarseMaps cm{};
    std::vector<int32_t> h_mortar_idx;     // per interface nu_c local ids
    std::vector<int64_t> h_iface_hoff;
    std::vector<double> h_H;
    std::vector<int32_t> h_corr_grains;

    // grains
    DenseSet gset;
    std::vector<int32_t> gm_grain, gm_ncol, gm_ntc, gm_k, gm_corr;
    std::vector<int64_t> gm_roff, gm_ytoff, gm_xtoff, gm_koff, gm_coff;
    int64_t gcol_len = 0;
    GrainGather gg{};
    AbarWork *d_abar = nullptr;
    int64_t n_abar = 0;
    int64_t *d_g_slot_dof = nullptr;   // grain vector slot -> dof
    int64_t *d_g_dof_slot = nullptr;   // dof -> grain vector slot
    int64_t *d_gcol_upos = nullptr;    // grain column slot -> coarse vector position
    // Y = W R, X = W^T Y, K = Y^T Y, XT; or, by substitution (basis_subst),
    // K = Y^T Y here and the backward rows of X and XT in basis_x_prog, the
    // forward rows of Y having run in the grain factorisation's steps
    std::vector<Launch> basis_prog, basis_x_prog;
    bool basis_subst = false;
    int64_t negi_off = -1;             // a -I tile in the FP64 arena (substitution terms)
    Range gemv_XT, gemv_X;
    std::vector<int64_t> pad_ones_g;   // identity on padded diagonals
    int64_t *d_pad_g = nullptr;
    // (offset, length) runs of the grain and contact-grid tiles inside the
    // tile envelope, cleared before each gather (the tiles outside it are
    // zeroed once and never written); empty: clear the whole region
    std::vector<int64_t> zero_g, zero_c;
    int64_t *d_zero_g = nullptr, *d_zero_c = nullptr;

    // contacts
    DenseSet cset;
    ContactGather cg{};
    int64_t n_citems = 0;
    int64_t *d_c_slot_dof = nullptr;
    int64_t *d_c_dof_ptr = nullptr;
    int64_t *d_c_dof_slot = nullptr;
    std::vector<int64_t> pad_ones_c;
    int64_t *d_pad_c = nullptr;
    int64_t c_stage_base = 0;          // fp64 staging region (reduced-precision mode)
    int64_t *d_c_aoff_stage = nullptr;

    // coarse
    CoarseMF mf;
    int64_t cvec_len = 0;
    double *pair_vals = nullptr;
    int64_t n_pair_vals = 0;
    std::vector<CoarsePair> h_pairs;
    CoarsePair *d_pairs = nullptr;
    int64_t n_pairs = 0;
    CoarseEdge *d_edges = nullptr;
    CoarseKRef *d_krefs = nullptr;
    int64_t *d_corr_koff = nullptr;

    // arenas
    double *ar64 = nullptr;
    int64_t ar64_n = 0;
    float *ar32 = nullptr;
    int64_t ar32_n = 0;
    uint16_t *arbf = nullptr;
    int64_t arbf_n = 0;
    TaskLists tl64, tl32;
    TaskLists tlbf;   // bfloat16 operands, FP32 results (S of the reduced-precision inverse form)
    // learned-basis surrogate inputs (host copies kept by the plan)
    std::vector<int32_t> sg_xyz;                 // [3 n_nodes] lattice coordinates
    std::vector<float> sg_logtr, sg_fill;        // per node: log trace of A_vv, stored blocks / 27
    std::vector<int64_t> sg_gnodes_ptr;          // per grain matrix: interior nodes (ascending)
    std::vector<int32_t> sg_gnodes;
    std::vector<int64_t> sg_adj_ptr;             // per grain matrix: adjacent interfaces, ascending,
    std::vector<int32_t> sg_adj, sg_lcol;        //   and the first local column of each
    std::vector<int32_t> sg_iface_nu;
    std::vector<int64_t> sg_iface_ptr;
    std::vector<int32_t> sg_iface_nodes;
    bool sg_ready = false;                       // device sample tables built
    struct Scratch {                             // grown on demand, freed with the handle
        void *p = nullptr;
        size_t cap = 0;
        void *get(size_t bytes) {
            if (bytes > cap) {
                if (p) (void)hipFree(p);
                p = nullptr;
                cap = 0;
                if (hipMalloc(&p, bytes) != hipSuccess) fail(HPLMM_E_OOM, "hipMalloc failed");
                cap = bytes;
            }
            return p;
        }
        ~Scratch() {
            if (p) (void)hipFree(p);
        }
    };
    Scratch sg_x, sg_y, sg_z, sg_norms, sg_tasks, sg_pairs, sg_copy, sg_cnt, sg_part, sg_meta;
    int64_t sg_total = 0;                        // (grain, interface, mortar) samples
    std::vector<int32_t> sg_s_m, sg_s_c, sg_s_a; // host copies of the sample list
    sg::SampleArgs sg_args{};
    GemvTask *d_vtasks = nullptr;
    int64_t gemv_part_len = 0;          // split-row partial sums (doubles)
    double *d_gemv_part = nullptr;
    // when set, the coarse sweeps' split rows use this instead of
    // d_gemv_part (the allocation-free application)
    double *split_part = nullptr;
    GemvPair *d_vpairs = nullptr;
    std::vector<GemvTask> vtasks;
    std::vector<GemvPair> vpairs;
    // symmetric smoother (inverse form): pairs of its row tasks (in vtasks),
    // the row sums of the transposed products, and their partial buffer
    int32_t smoother_form = HPLMM_SMOOTHER_FACTORS;
    std::vector<SymPair> spairs;
    std::vector<SymReduce> rtasks;
    SymPair *d_spairs = nullptr;
    SymReduce *d_rtasks = nullptr;
    int64_t sym_part_len = 0;
    double *d_sym_part = nullptr;
    int64_t grain_region_zero_n = 0;   // elements zeroed before each set-up

    // vectors
    double *gx = nullptr, *gt = nullptr, *gy = nullptr;   // grain local
    double *gc_t = nullptr, *gc_u = nullptr;               // grain columns
    double *cx = nullptr, *ct = nullptr, *cy = nullptr;   // contact local
    double *sf = nullptr, *st = nullptr, *su = nullptr;   // coarse
    double *z1 = nullptr, *z2 = nullptr, *r1 = nullptr, *r2 = nullptr, *tmpN = nullptr;
    double *corr_d = nullptr;
    int32_t *d_flag = nullptr;

    // Krylov workspace
    int32_t kr_restart = 0;
    double *V = nullptr, *Z = nullptr, *w = nullptr, *part = nullptr, *hbuf = nullptr, *h2 = nullptr;
    // HIP graphs of the Arnoldi steps (one per step index j of the restart
    // cycle), captured on an internal stream and replayed on the caller's; rebuilt
    // when the Krylov buffers change
    std::vector<TuneRecord> tune_log;   // launches chosen by hplmm_autotune (empty: defaults)
    // the contact-grid factorisation runs beside the grain and coarse stages on
    // its own stream, with its own split-task scratch when it shares tl64
    hipStream_t side = nullptr;
    hipEvent_t side_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    void *d_part_side = nullptr;
    bool use_graphs = true;
    hipStream_t gstream = nullptr;
    std::vector<hipGraphExec_t> arnoldi_graphs;
    const double *graph_key_V = nullptr;
    void drop_graphs() {
        for (hipGraphExec_t g : arnoldi_graphs)
            if (g) (void)hipGraphExecDestroy(g);
        arnoldi_graphs.clear();
        graph_key_V = nullptr;
    }
    double *ydev = nullptr;
    int32_t kr_blocks = 0;
    // pinned host copies of the last two steps' Hessenberg columns and the
    // events that mark them ready: step j + 1 is queued before the host
    // reads step j's column (one-step lookahead)
    double *hcol_host = nullptr;
    hipEvent_t hcol_ev[2] = {nullptr, nullptr};

    // the method's own work (unpadded sizes, each operator once), the figures
    // rooflines are stated against: set-up flops {grains: Cholesky N^3/3, two
    // triangular solves with the k+1 basis and correction columns 2 N^2 (k+1),
    // Galerkin block 2 N k^2; contact grids n^3/3; coarse fronts d^3/3 + d^2 u
    // + d u^2; total}, and the flops the set-up's tile tasks issue (64x64 tiles
    // with padding, the explicit inverses and S = W^T W included) {grains,
    // contact grids, coarse, total}
    double method_setup_flops[4] = {0, 0, 0, 0};
    double issued_setup_flops[4] = {0, 0, 0, 0};
    // bytes one application of M^-1 needs, each operator's stored triangle or
    // block read once: {smoother operators (grain + contact, as applied in the
    // chosen form and precision), restriction + prolongation, coarse sweeps,
    // fine products (two), whole application}
    double method_apply_bytes[5] = {0, 0, 0, 0, 0};

    // timings
    double t_setup_ms[4] = {0, 0, 0, 0};
    double t_ml_ms = 0.0, t_mg_ms = 0.0;   // the paper's T_ML and T_MG of the last set-up
    Profiler prof;
    double apply_bytes = 0.0, spmv_bytes = 0.0;
    // matrix-free fine operator (hplmm_set_voxel_operator): used by every SpMV
    // when on; the assembled figures are kept to switch back
    bool vop_on = false;
    VoxelGrid vop{};
    const int32_t *vop_xyz = nullptr;
    const double *vop_K = nullptr;
    double spmv_bytes_assembled = -1.0, apply_bytes_assembled = -1.0;

    template <class T>
    T *dalloc(int64_t n) {
        if (n <= 0) n = 1;
        void *p = nullptr;
        if (hipMalloc(&p, sizeof(T) * (size_t)n) != hipSuccess) fail(HPLMM_E_OOM, "hipMalloc failed");
        allocs.push_back(p);
        dev_bytes += (int64_t)(sizeof(T) * (size_t)n);
        return (T *)p;
    }
    template <class T>
    T *upload(const std::vector<T> &v, hipStream_t s) {
        T *p = dalloc<T>((int64_t)v.size());
        if (!v.empty() && hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s) != hipSuccess)
            fail(HPLMM_E_HIP, "hipMemcpyAsync failed");
        return p;
    }
    ~Handle() {
        drop_graphs();
        for (hipEvent_t e : hcol_ev)
            if (e) (void)hipEventDestroy(e);
        if (hcol_host) (void)hipHostFree(hcol_host);
        if (gstream) (void)hipStreamDestroy(gstream);
        for (hipEvent_t e : side_ev)
            if (e) (void)hipEventDestroy(e);
        if (side) (void)hipStreamDestroy(side);
        for (hipEvent_t e : prof.pool) (void)hipEventDestroy(e);
        for (void *p : allocs) (void)hipFree(p);
    }
};

// plan.cpp
void build_plan(Handle &h, const hplmm_system &sys, const hplmm_partition &part, const hplmm_mortar &mort,
                const hplmm_options &opt, hipStream_t s, bool dry_run);
std::vector<int32_t> place_mortars(const int32_t *xyz, int32_t N, int32_t n);
enum BasisParts { BP_Y = 1, BP_X = 2, BP_K = 4, BP_XT = 8, BP_ALL = 15 };
void append_basis_program(Handle &h, TaskLists &tl, const std::vector<int64_t> &ms, std::vector<Launch> &prog,
                          int parts);
void split_program(std::vector<Launch> &prog, TaskLists &tl);
void fill_flops(std::vector<Launch> &prog, const TaskLists &tl);
// sg_capi.cpp
void sg_build_sample_tables(Handle &h, hipStream_t s);
// capi.cpp: the preconditioner application behind hplmm_apply
void apply_op(Handle &h, int32_t which, const double *r, double *z, hipStream_t s);
// noalloc.hip: device address of the library's static split-row scratch on
// device dev, which must be current (resolved once per device)
void *static_scratch_address(int dev);

}  // namespace hplmm

struct hplmm_handle {
    hplmm::Handle h;
};

struct hplmm_sg_net;
namespace hplmm {
void sg_net_forward(hplmm_sg_net *net, const float *x, int32_t n, float *y, hipStream_t s);
int32_t sg_net_max_batch(const hplmm_sg_net *net);
bool sg_net_is_basis_net(const hplmm_sg_net *net);
}  // namespace hplmm
