/*
 * hplmm.h -- C ABI of the MI355X hPLMM library (libhplmm.so).
 *
 * The library solves the displacement-form linear-elastic system
 *     A x = b                                               (paper Eq. 4)
 * assembled with trilinear (Q1) hexahedra on a voxel grid (Sec. 2), with
 * right-preconditioned flexible GMRES and the algebraic hPLMM preconditioner
 *     M^-1 = M_G^-1 + M_L^-1 (I - A M_G^-1)                  (Eq. 16)
 * whose coarse part M_G^-1 = P^ (P^T A P^)^-1 P^T, P^ = W Q P (Eqs. 18-24)
 * is built from per-grain shape and correction vectors and Gaussian mortars
 * (Eqs. 7-8), and whose smoother M_L = M_CG is the contact-grain additive
 * Schwarz smoother (Eqs. 25-26).
 *
 * Conventions shared by every entry point:
 *  - Nodes are the free FEM nodes (nodes touched by a solid voxel that are
 *    not on the clamped plane z = 0), numbered 0..n_nodes-1.  Degrees of
 *    freedom are node-major: dof 3*v + c, c = x, y, z.  Vectors have 3*n_nodes
 *    float64 entries.
 *  - "host" arrays are ordinary CPU memory owned by the caller unless stated;
 *    the library copies what it keeps.  "device" arrays are HIP device memory
 *    (e.g. PyTorch CUDA tensors on ROCm) owned by the caller.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Device work is enqueued on that stream.
 *  - Every function returns an hplmm_status; errors never unwind across the
 *    ABI.  hplmm_last_error() gives a text message for the calling thread.
 *  - A handle is not thread safe; distinct handles are independent.
 */
#ifndef HPLMM_H
#define HPLMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hplmm_status;
#define HPLMM_OK                 0
#define HPLMM_NOT_CONVERGED      1   /* solve hit maxit; x holds the last iterate   */
#define HPLMM_E_ARG             -1   /* invalid argument, size or layout            */
#define HPLMM_E_PARTITION       -2   /* partition does not cover the nodes, or two
                                        grains' interiors are coupled by A          */
#define HPLMM_E_NOT_SPD         -3   /* a local or coarse Cholesky pivot was <= 0    */
#define HPLMM_E_SINGULAR_COARSE -4   /* coarse correction pivot b_i^T c_i <= 0       */
#define HPLMM_E_HIP             -5   /* a HIP runtime call failed                    */
#define HPLMM_E_OOM             -6   /* device allocation failed                     */
#define HPLMM_E_NONFINITE       -7   /* NaN/Inf in a Krylov quantity                 */
#define HPLMM_E_STATE           -8   /* call out of order (e.g. apply before setup)  */

typedef struct hplmm_handle hplmm_handle;

/* ---------------------------------------------------------------------------
 * Problem description (host side, no GPU needed).
 * ------------------------------------------------------------------------- */

/* Assembled fine system, block-sparse with 3x3 blocks (paper Eq. 4).
 * row_ptr[n_nodes+1] (int64), col_idx[nnzb] (int32, ascending within each
 * row, pattern symmetric), val[9*nnzb] row-major 3x3 blocks (float64).
 * rhs[3*n_nodes]: load vector b.  node_xyz[3*n_nodes]: integer lattice
 * coordinates (i, j, k) of every node.  dof_fixed[3*n_nodes] (uint8, may be
 * NULL): nonzero marks a constrained degree of freedom (a Dirichlet row of
 * Eq. 2 with zero prescribed displacement, e.g. a roller); hplmm_plan then
 * works on the matrix with that dof's row and column replaced by the identity's
 * and on the load with a zero there, so the solution is 0 at every
 * constrained dof (the plane z = 0 of hplmm_assemble_voxels is clamped by
 * elimination instead and needs no flags).  When returned by
 * hplmm_assemble_voxels the arrays are owned by the library (dof_fixed NULL)
 * and released with hplmm_system_free; when passed in, they are the
 * caller's and copied by hplmm_plan. */
typedef struct hplmm_system {
    int64_t n_nodes;
    int64_t nnzb;
    int64_t *row_ptr;
    int32_t *col_idx;
    double  *val;
    double  *rhs;
    int32_t *node_xyz;
    const uint8_t *dof_fixed;
} hplmm_system;

/* Decomposition into grain grids, contact interfaces and contact grids
 * (Sec. 3.1-3.2).  n_nodes must equal the system's.  node_grain[n_nodes]: grain id of a grain-interior node, or
 * -1 for an interface node.  Interfaces as CSR: iface_ptr[n_ifaces+1],
 * iface_nodes[...] (ascending node ids).  Contact grids as CSR:
 * contact_ptr[n_contacts+1], contact_nodes[...] (ascending).  Every node is
 * in exactly one grain interior or one interface.  Library-owned when
 * returned by hplmm_partition_from_voxels (free with hplmm_partition_free). */
typedef struct hplmm_partition {
    int64_t  n_nodes;
    int32_t  n_grains;
    int32_t *node_grain;
    int32_t  n_ifaces;
    int64_t *iface_ptr;
    int32_t *iface_nodes;
    int32_t  n_contacts;
    int64_t *contact_ptr;
    int32_t *contact_nodes;
} hplmm_partition;

/* Assemble the Q1 stiffness matrix and load of a voxel solid (Sec. 2,
 * Eqs. 1-4).  solid[nx*ny*nz] (uint8, x fastest), E[nx*ny*nz] Young's modulus
 * per voxel (ignored on void), nu Poisson ratio, traction[3] the uniform
 * traction on the top face z = nz of the top solid layer (consistent load,
 * a quarter per face node).  Voxel edge length 1; the plane z = 0 is clamped.
 * Host only.  On error *out is zeroed. */
hplmm_status hplmm_assemble_voxels(int32_t nx, int32_t ny, int32_t nz,
                                   const uint8_t *solid, const double *E, double nu,
                                   const double *traction, hplmm_system *out);
void hplmm_system_free(hplmm_system *sys);

/* Classify nodes and build interfaces and contact grids from a voxel
 * labelling (Sec. 3.1).  voxel_label[nx*ny*nz]: grain id in [0, n_labels)
 * for solid voxels (ignored on void).  A node whose touching solid voxels
 * carry one label is interior to that grain; otherwise it is an interface
 * node, and an interface is a connected set (two nodes connect when both are
 * corners of one solid voxel) of interface nodes with the same set of touching
 * labels.  Interfaces are numbered by smallest node id.  Contact grid c holds
 * every node within Chebyshev lattice distance w_zeta of interface c (the
 * dilation of Sec. 3.1).  Host only. */
hplmm_status hplmm_partition_from_voxels(int32_t nx, int32_t ny, int32_t nz,
                                         const uint8_t *solid, const int32_t *voxel_label,
                                         int32_t n_labels, int32_t w_zeta,
                                         hplmm_partition *out);
void hplmm_partition_free(hplmm_partition *part);

/* Mortar space (Sec. 3.3): n = mortar nodes per interface (n = 1 is PLMM),
 * beta = Gaussian spread (Eq. 8; the paper uses 4), kind = the mortar
 * functions:
 *   HPLMM_MORTAR_GAUSSIAN   Gaussian weights normalised to a partition of
 *                           unity, acting alike on x, y, z (Eq. 8);
 *   HPLMM_MORTAR_ALGEBRAIC  algebraic mortars (Eq. 9 in the algebraic form
 *                           that follows Eq. 22): column (node i, component g)
 *                           is 1 at that dof, 0 at the other mortar-node dofs
 *                           and -(A_FF)^-1 A_F,(i,g) on the remaining dofs F
 *                           of the interface, from the interface block of the
 *                           system matrix (computed by hplmm_plan; beta unused;
 *                           the learned surrogate needs Gaussian mortars). */
#define HPLMM_MORTAR_GAUSSIAN   0
#define HPLMM_MORTAR_ALGEBRAIC  1
typedef struct hplmm_mortar {
    int32_t n;
    double  beta;
    int32_t kind;
} hplmm_mortar;

/* Smoother precision: 64 = float64; 32 = float32 smoother operators; 16 =
 * bfloat16 smoother operators.  The coarse space (basis, coarse operator,
 * coarse solve) and the Krylov solver are float64 in every mode.
 * coarse_leaf_dofs: the nested dissection of the coarse operator stops at
 * subsets of at most this many dofs (0 = the default, 192); larger leaves
 * give fewer front levels (fewer launches per coarse solve) and larger dense
 * leaf fronts.
 * smoother_form: how the smoother applies the local inverses A_g^-1 and
 * A_zeta^-1 of Eqs. 25-26 (the same operator either way, up to rounding):
 *   HPLMM_SMOOTHER_FACTORS  y = W^T (W x) with W = L^-1: two passes, each over
 *                           the lower tiles of the block.  At smoother_precision
 *                           32 / 16 the grain W is the float64 one rounded to
 *                           float32 / bfloat16, and the contact grids are
 *                           factored and inverted in float32 on the matrix cores
 *                           (float32 accumulation), their W rounded to the
 *                           storage precision;
 *   HPLMM_SMOOTHER_INVERSE  y = S x with S = W^T W formed in the set-up (one
 *                           more batched tile product and one more arena
 *                           region per set): one pass over the lower tiles of
 *                           S, each off-diagonal tile serving S_ij x_j and
 *                           S_ij^T x_i, then a short sum of the transposed
 *                           products per tile row.  Half the smoother's HBM
 *                           reads.  At smoother_precision 32 / 16 every block is
 *                           factored and inverted in float64, W is rounded to
 *                           float32 / bfloat16 (Wp), and S = Wp^T Wp is formed
 *                           from the rounded values on the matrix cores
 *                           (float32 / bfloat16 operands, float32
 *                           accumulation) and kept in float32: the Gram matrix
 *                           of Wp, positive definite however coarse the
 *                           rounding;
 *   HPLMM_SMOOTHER_AUTO (0) the inverse form. */
#define HPLMM_SMOOTHER_AUTO     0
#define HPLMM_SMOOTHER_FACTORS  1
#define HPLMM_SMOOTHER_INVERSE  2
typedef struct hplmm_options {
    int32_t smoother_precision;
    int32_t coarse_leaf_dofs;
    int32_t smoother_form;
} hplmm_options;

/* Place the mortar nodes of one interface (Sec. 3.3, Eq. 7): xyz[3*N] lattice
 * coordinates of its nodes in interface order; writes nu = min(n, N) node
 * indices (into 0..N-1) to idx_out.  Host only; exposed for testing. */
hplmm_status hplmm_place_mortars(const int32_t *xyz, int32_t N, int32_t n, int32_t *idx_out);

/* ---------------------------------------------------------------------------
 * Preconditioner and solver (device).
 * ------------------------------------------------------------------------- */

/* Symbolic phase: validate the system and partition, place mortars and
 * compute Gaussian weights (Eqs. 7-8), decide the correction columns from
 * the load (a grain whose load is identically zero gets none), build the
 * device data layout and the launch plans, and upload A, b and all index
 * maps to the current device.  Host arrays are copied and may be released
 * afterwards.  b may be NULL (no correction columns).  The returned handle
 * owns all device memory until hplmm_destroy. */
hplmm_status hplmm_plan(const hplmm_system *sys, const hplmm_partition *part,
                        const hplmm_mortar *mortar, const hplmm_options *opt,
                        void *stream, hplmm_handle **out);

/* Host-only dry run of hplmm_plan: the same validation and planning, then a
 * bounds check of every launch task list and index map against the buffers
 * they address, without touching a device.  sizes (may be NULL) receives
 * int64[16] = {n_nodes, nnzb, n_grains, n_ifaces, n_contacts, n_mortar_dofs,
 * n_corr, n_coarse, grain_mats, f64 arena elements, f32 arena elements, bf16
 * arena elements, f64 tile tasks, coarse fronts, coarse levels, largest front
 * (dofs)}. */
hplmm_status hplmm_plan_check(const hplmm_system *sys, const hplmm_partition *part,
                              const hplmm_mortar *mortar, const hplmm_options *opt, int64_t *sizes);

/* Numeric set-up on the device (the paper's T_MG + T_ML): gather grain,
 * contact and coupling blocks; batched Cholesky and triangular inversion of
 * grain blocks A_gi and contact blocks; basis X_i = A_gi^-1 [-Abar_gi | b_gi]
 * (Eqs. 23-24); Galerkin coarse operator P^T A P^ (Eq. 18) and its
 * factorisation.  The contact-grid blocks are factored on an internal stream
 * that is forked from `stream` and joined back into it.  Returns after one
 * final synchronising check of the pivot flags (reported as HPLMM_E_NOT_SPD /
 * HPLMM_E_SINGULAR_COARSE). */
hplmm_status hplmm_setup(hplmm_handle *h, void *stream);

/* z = Op r for r, z device vectors of 3*n_nodes float64 (must not alias).
 * which: 0 = M^-1 (Eq. 16), 1 = M_G^-1 (Eq. 18), 2 = M_CG^-1 (Eq. 25),
 *        3 = M_zeta^-1, 4 = M_g^-1 (Eq. 26).  Asynchronous on `stream`. */
hplmm_status hplmm_apply(hplmm_handle *h, int32_t which, const double *r_dev,
                         double *z_dev, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * z = Op r as hplmm_apply (same which, same kernels, same results bit for
 * bit), but the application's scratch -- the partial sums of the coarse
 * sweeps' split rows -- is taken from a static 8 MiB device buffer of the
 * library instead of the handle's, and the call allocates nothing: no device
 * memory, no events (the built-in profiler does not see its launches).  Every
 * partial sum is written before it is read within the call, so the buffer
 * needs no clearing.  Each device holds one such buffer until the process ends,
 * shared by every call on that device: calls that overlap on one device (two
 * streams, two threads, two handles) race and must be ordered by the caller.
 * The other per-handle buffers (local vectors, the symmetric smoother's
 * per-tile sums) are the handle's, allocated by hplmm_plan, as for
 * hplmm_apply.  Errors: E_ARG for NULL or aliased vectors, which outside
 * 0..4, a handle planned on another device than the current one, or a plan
 * whose split rows need more than the buffer (the message gives the bytes);
 * E_STATE before set-up.  Query 12 gives the split-row scratch a plan needs:
 * int64[1] = {partial sums (doubles)}. */
hplmm_status hplmm_apply_noalloc(hplmm_handle *h, int32_t which, const double *r_dev, double *z_dev,
                                 void *stream);

/* y = A x (device vectors, must not alias).  Asynchronous. */
hplmm_status hplmm_spmv(hplmm_handle *h, const double *x_dev, double *y_dev, void *stream);

/* Solve A x = b with right-preconditioned flexible GMRES(restart) and M.
 * b_dev: right-hand side (device); x_dev: initial guess on entry (device),
 * solution on exit.  Stops when the true residual |b - A x| / |b| < rtol
 * (checked whenever the Arnoldi estimate drops below rtol and at every
 * restart) or after maxit Arnoldi steps.  fixed_iters > 0 runs exactly that
 * many steps and forms x.  Synchronises with the host once per step.
 * info (may be NULL) receives the counts, times and the residual history
 * (res_hist: caller buffer of res_hist_cap doubles, may be NULL). */
typedef struct hplmm_solve_info {
    int32_t iters;
    double  rel_res_true;
    double  t_solve_ms;      /* the paper's T_sol (host clock around the solve) */
    double *res_hist;
    int32_t res_hist_cap;
    int32_t res_hist_len;
    double  t_ml_ms;         /* T_ML of the last set-up: grain factorisations, contact
                                grids and the grain inverse S (HIP events) */
    double  t_mg_ms;         /* T_MG of the last set-up: basis, coarse operator and its
                                factorisation (HIP events); T_ML and T_MG overlap on the
                                device, so their sum exceeds the set-up's wall time */
} hplmm_solve_info;

hplmm_status hplmm_solve(hplmm_handle *h, const double *b_dev, double *x_dev, double rtol,
                         int32_t restart, int32_t maxit, int32_t fixed_iters,
                         hplmm_solve_info *info, void *stream);

/* Introspection for tests and benchmarks.  what:
 *   0 sizes: int64[16] = {n_nodes, nnzb, n_grains, n_ifaces, n_contacts,
 *            n_mortar_dofs, n_corr, n_coarse, grain_mats, max_grain_dofs,
 *            max_contact_dofs, sell_slices, sell_padded_blocks, coarse_fronts,
 *            coarse_levels, max_front_dofs}
 *   1 mortar node ids: int32 per interface, concatenated in interface order
 *            (nu_c entries each, local indices into the interface's nodes)
 *   2 mortar blocks: float64 per interface, row-major; Gaussian: H_c
 *            (N_c x nu_c), algebraic: the 3 N_c x 3 nu_c block of Q^o (rows
 *            3 v + g, columns 3 i + g')
 *   3 correction grains: int32[n_corr] grain ids, ascending
 *   4 coarse matrix: float64 n_coarse x n_coarse row-major (after setup):
 *            mortar block then the correction diagonal
 *   5 setup phase times in ms: double[4] = {grains, contacts, coarse, total};
 *            the contact grids are set up on an internal stream beside the
 *            grains and the coarse operator, so total (the wall time of the
 *            set-up) is less than the sum; in the inverse smoother form the
 *            grain inverse S = W^T W follows the contact grids on that stream
 *            and is counted in none of the first three
 *   6 device bytes held: int64[1]
 *   7 profiler totals (see hplmm_profile)
 *   8 algorithmic bytes: double[2] = {one application of M^-1, one SpMV}
 *   9 coarse solve structure: double[5 * levels], per front level (0 = root)
 *            {fronts, forward work-groups, forward bytes, backward
 *            work-groups, backward bytes} (with the current launch shapes)
 *  10 tuning records: double[7 * k], one per tuned launch {kind, index,
 *            variant, target work-groups, waves, default us, chosen us}
 *            (see hplmm_autotune; empty with the default shapes); the
 *            smoother launches are listed as grain W, grain W^T, contact W,
 *            contact W^T, X^T, X in the factor form and grain S, contact S,
 *            X^T, X in the inverse form
 *  11 smoother form in use: int32[1] (HPLMM_SMOOTHER_FACTORS or _INVERSE)
 *  12 split-row scratch of the coarse sweeps: int64[1] = {partial sums
 *            (doubles)}
 *  13 the method's own work, from unpadded sizes: double[13] =
 *            {set-up flops: grains (N^3/3 Cholesky + 2 N^2 c triangular
 *            solves with the c = k (+1) basis and correction columns + 2 N k^2
 *            Galerkin block), contact grids (n^3/3), coarse fronts (d^3/3 +
 *            d^2 u + d u^2 for d own, u boundary dofs), total;
 *            flops the set-up's 64x64 tile tasks issue (padding, explicit
 *            inverses W = L^-1 and S = W^T W included): grains, contact grids,
 *            coarse, total;
 *            bytes of one M^-1 application with every operator's stored
 *            triangle or block read once: smoother operators (as applied in
 *            the chosen form and precision), restriction + prolongation,
 *            coarse sweeps, the two residual products, whole application}
 * host_out receives at most cap_bytes bytes; *needed_bytes gets the size. */
hplmm_status hplmm_query(hplmm_handle *h, int32_t what, void *host_out, int64_t cap_bytes,
                         int64_t *needed_bytes);

/* Launch-shape autotuning of the solve phase (after hplmm_setup).  The
 * GEMV launches of M^-1 are timed on this problem's own operators (reps
 * back-to-back launches, best of three, events on stream; the call
 * synchronises) and each keeps its fastest shape:
 *   kind 0 / 1, index l: the forward / backward coarse sweep at front level l,
 *     variants = its rows as planned (variant 0: split over about 256
 *     work-groups when the level has fewer than 128 rows, else unsplit),
 *     unsplit, or split over about 256, 512, 1024, 2048 work-groups;
 *   kind 2, index 0..5: grain W, grain W^T, contact W, contact W^T, X^T, X
 *     products (variant 0 only);
 * each at 4 or 16 wavefronts per work-group.  A different shape changes the
 * order in which partial sums are added (results agree to rounding; a fixed
 * set of shapes always gives the same bits).  The coarse front vectors are
 * zeroed.  Query 10 returns the choices with the timings; E_STATE before
 * set-up; reps in 1..1000. */
hplmm_status hplmm_autotune(hplmm_handle *h, int32_t reps, void *stream);

/* Pin launch shapes without timing: rec holds n records {kind, index,
 * variant, waves} (int32, as in query 10); launches not named keep their
 * default shape, n = 0 restores every default.  E_ARG on a kind, index,
 * variant or waves (4 or 16) out of range, in which case the defaults are
 * restored.  Synchronises the device. */
hplmm_status hplmm_set_tuning(hplmm_handle *h, const int32_t *rec, int64_t n);

/* Matrix-free fine operator for problems assembled from a voxel grid (the
 * grid, E and nu that hplmm_assemble_voxels was given): every later product
 * with A (hplmm_spmv, the preconditioner's residuals, the solver) sums
 * E_e Khat(nu) x over each free node's solid voxels instead of streaming the
 * assembled 3x3 blocks (Eq. 4).  The set-up still uses the assembled matrix.
 * solid[nx*ny*nz] (uint8) and E[nx*ny*nz] are host arrays (copied).  The
 * call compares both operators on a seeded vector and fails with E_ARG,
 * leaving the assembled operator in use, if they differ by more than 1e-12
 * of max |A x| (a different grid, modulus or nu), and with E_ARG if the
 * system has constrained dofs (dof_fixed).  nx = ny = nz = 0 returns
 * to the assembled operator.  Synchronises stream; each call that turns the
 * operator on allocates its own device copies (held until hplmm_destroy);
 * captured solver graphs are dropped. */
hplmm_status hplmm_set_voxel_operator(hplmm_handle *h, int32_t nx, int32_t ny, int32_t nz,
                                      const uint8_t *solid, const double *E, double nu, void *stream);

/* HIP graphs for the solver (on by default): hplmm_solve captures each
 * Arnoldi step j of the restart cycle (M^-1 application, SpMV, the two
 * Gram-Schmidt passes, normalisation: kernel launches only) into a graph the
 * first time it runs (capture happens on an internal stream) and launches
 * the graph on the caller's stream from then on.  Graphs are rebuilt when the Krylov
 * buffers are reallocated and are not used while the profiler times a
 * solve-phase class (classes 2-7).  The
 * results are identical with graphs on and off.  on = 0 turns them off and
 * frees them. */
hplmm_status hplmm_use_graphs(hplmm_handle *h, int32_t on);

/* Built-in kernel profiler: when bit c of mask is set, HIP events are
 * recorded on the launch stream around every launch of kernel class c:
 *   0 set-up tile contractions, 1 diagonal-tile factorisations, 2 smoother
 *   GEMVs, 3 coarse-solve GEMVs, 4 restriction/prolongation GEMVs, 5 fine
 *   SpMV, 6 whole applications of M^-1, 7 sums of the transposed products
 *   of the symmetric smoother (inverse form).
 * Query 7 returns double[3*8] = per class {launches, total ms, total
 * algorithmic units} (flops for class 0, tiles for 1, bytes otherwise) over
 * all launches since the last hplmm_profile call, which clears them.  mask = 0 turns the
 * profiler off (no events are recorded). */
hplmm_status hplmm_profile(hplmm_handle *h, int32_t mask);

void        hplmm_destroy(hplmm_handle *h);
const char *hplmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HPLMM_H */
