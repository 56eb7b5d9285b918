// Post-processing of a displacement solution on its voxel grid: stresses at
// voxel centroids for the error metric of Eq. 28.
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
};

// sigma_t[v] = max shear stress, uc[3v + c] = centroid displacement of voxel v
// (zero on void voxels; uc may be null).
void launch_voxel_fields(const VoxelGrid &g, const double *x, double *sigma_t, double *uc, hipStream_t s);

}  // namespace hplmm
