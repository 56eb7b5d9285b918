/* Post-processing of libhplmm solutions on their voxel grid: the stresses
 * behind the first-pass error metric (Eq. 28, Sec. 5.1), which compares the
 * displacement u and the maximum shear stress sigma^t = (sigma_max -
 * sigma_min) / 2 (radius of the largest Mohr circle of the Hooke's-law stress,
 * Eqs. 1 and 3) of an approximate solution with those of the exact one.
 *
 * Errors follow hplmm.h (status codes, hplmm_last_error()).
 */
#ifndef HPLMM_POST_H
#define HPLMM_POST_H

#include "hplmm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Fields at the centroid of every voxel of an nx x ny x nz grid (x fastest,
 * unit voxels, one Q1 element per solid voxel):
 *   sigma_t[v]        maximum shear stress of the element stress at the
 *                     centroid, sigma = lambda tr(eps) I + 2 mu eps with the
 *                     voxel's E and nu (Eq. 3);
 *   u_centroid[3v+c]  mean of the eight corner displacements (may be NULL).
 * Void voxels get zeros.  Device arrays: solid[nx*ny*nz] (uint8, 1 = solid),
 * E[nx*ny*nz], lat2node[(nx+1)*(ny+1)*(nz+1)] = free node id of each lattice
 * point or -1 (clamped or unused: zero displacement; ids outside
 * [0, n_nodes) also read as zero), x[3*n_nodes] the displacement (node-major,
 * as hplmm_solve returns it).  Outputs are overwritten.  E_ARG on empty or
 * oversized grids (more than 2^31 voxels), nu outside (-1, 0.5) or NULL
 * required pointers.  Asynchronous on stream. */
hplmm_status hplmm_voxel_fields(int32_t nx, int32_t ny, int32_t nz, const uint8_t *solid, const double *E, double nu,
                                const int32_t *lat2node, int64_t n_nodes, const double *x, double *sigma_t,
                                double *u_centroid, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HPLMM_POST_H */
