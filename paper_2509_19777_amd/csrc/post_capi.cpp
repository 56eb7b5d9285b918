// C ABI of the post-processing kernels.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/hplmm_post.h"
#include "common.h"
#include "post.h"

using namespace hplmm;

extern "C" hplmm_status hplmm_voxel_fields(int32_t nx, int32_t ny, int32_t nz, const uint8_t *solid, const double *E,
                                           double nu, const int32_t *lat2node, int64_t n_nodes, const double *x,
                                           double *sigma_t, double *u_centroid, void *stream) {
    return guarded([&]() -> hplmm_status {
        if (nx < 1 || ny < 1 || nz < 1) fail(HPLMM_E_ARG, "grid dimensions must be positive");
        if ((int64_t)nx * ny * nz > ((int64_t)1 << 31)) fail(HPLMM_E_ARG, "more than 2^31 voxels");
        if (!(nu > -1.0 && nu < 0.5)) fail(HPLMM_E_ARG, "nu must lie in (-1, 0.5)");
        if (n_nodes < 0) fail(HPLMM_E_ARG, "n_nodes must be >= 0");
        if (!solid || !E || !lat2node || !sigma_t || (n_nodes > 0 && !x)) fail(HPLMM_E_ARG, "NULL array");
        const VoxelGrid g{nx, ny, nz, solid, E, nu, lat2node, n_nodes};
        launch_voxel_fields(g, x, sigma_t, u_centroid, (hipStream_t)stream);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) fail(HPLMM_E_HIP, std::string("voxel_fields launch: ") + hipGetErrorString(e));
        return HPLMM_OK;
    });
}
