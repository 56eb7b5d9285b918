// Kernels on a problem's voxel grid.
// * Stress recovery at voxel centroids (Hooke's law, Eqs. 1 and 3) and the
//   maximum shear stress (the Mohr-circle radius used by the error metric of
//   Eq. 28), one thread per voxel: the eight corner displacements give the
//   displacement gradient at the centroid of the unit Q1 cube, where every
//   shape-function derivative is +-1/4.
// * The matrix-free Q1 operator (Eq. 4 without the assembled blocks), one
//   thread per free node.
#include "post.h"

namespace hplmm {
namespace {

// Smallest and largest eigenvalue of a symmetric 3x3 matrix by cyclic Jacobi
// rotations (the two-sided symmetric Schur rotation of Golub and Van Loan,
// Matrix Computations, Sec. 8.5): each rotation zeroes a[p][q]; six sweeps
// take a 3x3 matrix to a diagonal within rounding.
__device__ void sym3_eig_range(double a[3][3], double &lo, double &hi) {
    for (int sweep = 0; sweep < 6; ++sweep) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int p = k == 2 ? 1 : 0, q = k == 0 ? 1 : 2, r = 3 - p - q;
            const double apq = a[p][q];
            if (apq == 0.0) continue;
            const double tau = (a[q][q] - a[p][p]) / (2.0 * apq);
            const double t = fabs(tau) > 1e150 ? 0.5 / tau : copysign(1.0, tau) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            const double arp = a[r][p], arq = a[r][q];
            a[p][p] -= t * apq;
            a[q][q] += t * apq;
            a[p][q] = a[q][p] = 0.0;
            a[r][p] = a[p][r] = c * arp - s * arq;
            a[r][q] = a[q][r] = s * arp + c * arq;
        }
    }
    lo = fmin(a[0][0], fmin(a[1][1], a[2][2]));
    hi = fmax(a[0][0], fmax(a[1][1], a[2][2]));
}

__global__ void __launch_bounds__(256) voxel_fields_kernel(VoxelGrid g, const double *__restrict__ x,
                                                           double *__restrict__ st, double *__restrict__ uc) {
    const int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    if (!g.solid[v]) {
        st[v] = 0.0;
        if (uc)
            for (int c = 0; c < 3; ++c) uc[3 * v + c] = 0.0;
        return;
    }
    const int64_t i = v % g.nx, j = (v / g.nx) % g.ny, k = v / ((int64_t)g.nx * g.ny);
    const int64_t NX = g.nx + 1, NY = g.ny + 1;
    double grad[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};   // grad[c][d] = du_c / dx_d
    double us[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int cx = a & 1, cy = (a >> 1) & 1, cz = (a >> 2) & 1;
        const int32_t node = g.lat2node[(i + cx) + NX * ((j + cy) + NY * (k + cz))];
        if (node < 0 || node >= g.n_nodes) continue;   // clamped or unused: zero displacement
        const double sx = cx ? 0.25 : -0.25, sy = cy ? 0.25 : -0.25, sz = cz ? 0.25 : -0.25;
        for (int c = 0; c < 3; ++c) {
            const double u = x[3 * (int64_t)node + c];
            us[c] += u;
            grad[c][0] += sx * u;
            grad[c][1] += sy * u;
            grad[c][2] += sz * u;
        }
    }
    const double E = g.E[v];
    const double lam = E * g.nu / ((1.0 + g.nu) * (1.0 - 2.0 * g.nu)), mu = E / (2.0 * (1.0 + g.nu));
    const double tr = grad[0][0] + grad[1][1] + grad[2][2];
    double s[3][3];
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) s[c][d] = mu * (grad[c][d] + grad[d][c]) + (c == d ? lam * tr : 0.0);
    double lo, hi;
    sym3_eig_range(s, lo, hi);
    st[v] = 0.5 * (hi - lo);
    if (uc)
        for (int c = 0; c < 3; ++c) uc[3 * v + c] = 0.125 * us[c];
}

// One thread per free node.  The moduli of its eight surrounding voxels are
// read once (zero for void or outside voxels); then for each of the 27
// neighbouring lattice nodes w the displacement x_w is read once and
// multiplied by the sum over the voxels holding both nodes of E_e times the
// 3x3 block of Khat that couples their corners.  Khat is staged in LDS.  The
// grids carry a halo, so no lookup needs a range test.
__global__ void __launch_bounds__(256) spmv_voxel_kernel(VoxelGrid g, const int32_t *__restrict__ xyz,
                                                         const double *__restrict__ Khat,
                                                         const double *__restrict__ x,
                                                         const double *__restrict__ r, double *__restrict__ y) {
    __shared__ double K[24 * 24];
    for (int e = threadIdx.x; e < 24 * 24; e += blockDim.x) K[e] = Khat[e];
    __syncthreads();
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= g.n_nodes) return;
    const int32_t i = xyz[3 * v], j = xyz[3 * v + 1], k = xyz[3 * v + 2];
    // padded grids: voxel (ex, ey, ez) at Ep[(ex + 1) + PX ((ey + 1) + PY (ez + 1))],
    // lattice point (a, b, c) at latp[(a + 1) + QX ((b + 1) + QY (c + 1))]; every
    // index below stays inside them, so all loads are issued without branches
    const int64_t PX = g.nx + 2, PY = g.ny + 2, QX = g.nx + 3, QY = g.ny + 3;
    double Ee[8];   // voxel (i - cx, j - cy, k - cz) holds this node at its corner e = cx + 2 cy + 4 cz
#pragma unroll
    for (int e = 0; e < 8; ++e)
        Ee[e] = g.Ep[(i - (e & 1) + 1) + PX * ((j - ((e >> 1) & 1) + 1) + PY * (int64_t)(k - ((e >> 2) & 1) + 1))];
    // the neighbours' displacements in groups of three offsets (one lattice
    // row q = (dy + 1) + 3 (dz + 1)), the next row's node numbers and
    // displacements loaded before the current row's products; the rows run as
    // a loop (not unrolled), so the compiler cannot hoist every row's loads at
    // once, and the in-element tests below are uniform branches
    double cur[9], nxt[9];
    auto load_row = [&](int q, double (&xg)[9]) {
        const int32_t *lrow = g.latp + i + QX * ((j + q % 3) + QY * (int64_t)(k + q / 3));
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int32_t wv = lrow[t];
            const bool ok = wv >= 0 && wv < g.n_nodes;
            const int64_t w = ok ? wv : v;   // a valid address either way
            xg[3 * t] = ok ? x[3 * w] : 0.0;
            xg[3 * t + 1] = ok ? x[3 * w + 1] : 0.0;
            xg[3 * t + 2] = ok ? x[3 * w + 2] : 0.0;
        }
    };
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    load_row(0, nxt);
#pragma unroll 1
    for (int q = 0; q < 9; ++q) {
#pragma unroll
        for (int c = 0; c < 9; ++c) cur[c] = nxt[c];
        if (q + 1 < 9) load_row(q + 1, nxt);
        const int oy = q % 3 - 1, oz = q / 3 - 1;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int ox = t - 1;
            const double x0 = cur[3 * t], x1 = cur[3 * t + 1], x2 = cur[3 * t + 2];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int cx = e & 1, cy = (e >> 1) & 1, cz = (e >> 2) & 1;
                const int bx = cx + ox, by = cy + oy, bz = cz + oz;
                if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;   // uniform
                const int b = bx + 2 * by + 4 * bz;
                const double *Kr = K + 3 * e * 24 + 3 * b;
                const double E = Ee[e];
                a0 += E * (Kr[0] * x0 + Kr[1] * x1 + Kr[2] * x2);
                a1 += E * (Kr[24] * x0 + Kr[25] * x1 + Kr[26] * x2);
                a2 += E * (Kr[48] * x0 + Kr[49] * x1 + Kr[50] * x2);
            }
        }
    }
    if (r) {
        y[3 * v] = r[3 * v] - a0;
        y[3 * v + 1] = r[3 * v + 1] - a1;
        y[3 * v + 2] = r[3 * v + 2] - a2;
    } else {
        y[3 * v] = a0;
        y[3 * v + 1] = a1;
        y[3 * v + 2] = a2;
    }
}

}  // namespace

void launch_spmv_voxel(const VoxelGrid &g, const int32_t *xyz, const double *Khat, const double *x, const double *r,
                       double *y, hipStream_t s) {
    if (g.n_nodes <= 0) return;
    hipLaunchKernelGGL(spmv_voxel_kernel, dim3((unsigned)((g.n_nodes + 255) / 256)), dim3(256), 0, s, g, xyz, Khat, x,
                       r, y);
}

void launch_voxel_fields(const VoxelGrid &g, const double *x, double *sigma_t, double *uc, hipStream_t s) {
    const int64_t nvox = (int64_t)g.nx * g.ny * g.nz;
    if (nvox <= 0) return;
    hipLaunchKernelGGL(voxel_fields_kernel, dim3((unsigned)((nvox + 255) / 256)), dim3(256), 0, s, g, x, sigma_t, uc);
}

}  // namespace hplmm
