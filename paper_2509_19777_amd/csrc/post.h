// Kernels on the voxel grid of a problem: stresses at voxel centroids for the
// error metric of Eq. 28, and the matrix-free fine operator.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hplmm {

struct VoxelGrid {
    int32_t nx, ny, nz;
    const uint8_t *solid;      // [nz][ny][nx]
    const double *E;           // [nz][ny][nx]
    double nu;
    const int32_t *lat2node;   // [(nz+1)(ny+1)(nx+1)] free node or -1
    int64_t n_nodes;
    // the same with a one-cell halo, so that every neighbour lookup of the
    // matrix-free operator is in range and needs no branch:
    const double *Ep;          // [(nz+2)(ny+2)(nx+2)] E on solid voxels, 0 on void and halo
    const int32_t *latp;       // [(nz+3)(ny+3)(nx+3)] free node or -1 (-1 on the halo)
};

// sigma_t[v] = max shear stress, uc[3v + c] = centroid displacement of voxel v
// (zero on void voxels; uc may be null).
void launch_voxel_fields(const VoxelGrid &g, const double *x, double *sigma_t, double *uc, hipStream_t s);

// Matrix-free y = A x (r == null) or y = r - A x with A the Q1 stiffness of
// the grid: every free node sums E_e Khat(nu) x over its (up to) eight solid
// voxels.  xyz[3 n_nodes]: lattice coordinates of the free nodes; Khat[24*24]:
// the unit-modulus element matrix, row-major, local node a at corner
// (a & 1, a >> 1 & 1, a >> 2 & 1), dof 3 a + c.
void launch_spmv_voxel(const VoxelGrid &g, const int32_t *xyz, const double *Khat, const double *x,
                       const double *r, double *y, hipStream_t s);

}  // namespace hplmm
