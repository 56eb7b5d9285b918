/*
 * hplmm_debug.h -- test hooks of libhplmm.
 *
 * These entry points exist so that tests can check single kernels of the
 * library (one 64x64 tile contraction, one diagonal-tile factorisation) and
 * the intermediate state of the set-up against an independent reference.
 * They are not needed to use the solver.  Same conventions as hplmm.h.
 */
#ifndef HPLMM_DEBUG_H
#define HPLMM_DEBUG_H

#include "hplmm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One tile task of the set-up contraction kernel on caller device buffers:
 * C (op)= alpha [P] sum_p op(A_p) op(B_p) with 64x64 column-major tiles.
 * A_dev, B_dev: npairs tiles each, consecutive; C_dev: one tile; P_dev: one
 * tile or NULL; flags: bit0 transpose A, bit1 transpose B, bit2 accumulate
 * into C, bit3 alpha = -1, bit4 left-multiply by P (C = alpha P S), bit5
 * right-multiply by P (C = ([C +] alpha S) P); bits 4 and 5 exclude each other
 * and need P.  npairs may be 0 only with bit5.  precision 64 or 32 selects
 * float64 or float32 tiles (all buffers of that type); precision 16 takes
 * bfloat16 A and B (their 16 bits), a float32 C and bits 0-3 only (the
 * bfloat16 matrix-core instruction with float32 accumulation). */
hplmm_status hplmm_debug_tile_gemm(int32_t precision, const void *A_dev, const void *B_dev, int32_t npairs,
                                   const void *P_dev, void *C_dev, int32_t flags, void *stream);

/* One diagonal-tile factorisation: A_dev (64x64 column-major; lower part
 * read) is overwritten by the Cholesky factor L of A - P P^T (zeros above),
 * W_dev gets L^-1 and Wt_dev gets L^-T.  P_dev is one 64x64 column-major tile
 * or NULL (then P = 0).  Returns HPLMM_E_NOT_SPD on a bad pivot. */
hplmm_status hplmm_debug_diag(int32_t precision, void *A_dev, const void *P_dev, void *W_dev, void *Wt_dev,
                              void *stream);

/* Bandwidth reference for measurements: a[i] = b[i] + scalar c[i], i < n,
 * on caller device arrays (float64, 16-byte aligned, a distinct from b and
 * c), launched on the stream without synchronising.  Moves 24 n bytes (two
 * reads, one write): the streaming-triad figure that HBM rates are compared
 * with beside the vendor peak. */
hplmm_status hplmm_stream_triad(double *a, const double *b, const double *c, double scalar, int64_t n,
                                void *stream);

/* Run the numeric set-up of a planned handle up to a stage and stop:
 *   stage 0: zero and gather grain blocks, coupling blocks and loads
 *   stage 1: + grain factorisation (Cholesky and inverse)
 *   stage 2: + basis products
 *   stage 3: full set-up (same as hplmm_setup).
 * Synchronises before returning. */
hplmm_status hplmm_debug_setup_stage(hplmm_handle *h, int32_t stage, void *stream);

/* Copy count elements starting at element offset off of an internal arena
 * (0 = float64, 1 = float32, 2 = bfloat16 bits) to host memory. */
hplmm_status hplmm_debug_read_arena(hplmm_handle *h, int32_t arena, int64_t off, int64_t count, void *host_out);

/* Layout of a planned handle for tests: int64 per grain matrix m (grain id,
 * dofs, tiles nt, columns ncol, column tiles ntc, A offset, W offset, Wt
 * offset, R offset, Y offset, K offset) -- 11 values per matrix.  The Wt
 * offset is -1 in the inverse smoother form, which stores no transposes. */
hplmm_status hplmm_debug_grain_layout(hplmm_handle *h, int64_t *out, int64_t cap);

/* Layout of the contact-grid blocks for tests: int64 per contact matrix m
 * (dofs n, tiles nt, arena holding its factor (0 = float64, 1 = float32), A/L
 * offset, W offset, Wt offset or -1 as for the grains) -- 6 values per
 * matrix, in contact-grid order.
 * Tiles are 64 x 64, column-major inside a tile, packed lower tiles (I, J),
 * I >= J, at I (I + 1) / 2 + J. */
hplmm_status hplmm_debug_contact_layout(hplmm_handle *h, int64_t *out, int64_t cap);

/* Host only: the per-interface mortar blocks that hplmm_plan would build (the
 * layout of query 2), concatenated in interface order, without touching the
 * device.  out receives at most cap doubles; *needed gets the total. */
hplmm_status hplmm_debug_mortar_blocks(const hplmm_system *sys, const hplmm_partition *part,
                                       const hplmm_mortar *mortar, double *out, int64_t cap, int64_t *needed);

#ifdef __cplusplus
}
#endif
#endif /* HPLMM_DEBUG_H */
