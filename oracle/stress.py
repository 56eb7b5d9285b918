"""Oracle: stress recovery and the first-pass error metric (Eq. 28).
TEST INFRASTRUCTURE ONLY: imported by tests/ and the variant study's checks,
never by the library.

The paper measures the first-pass solution M_G^-1 b (Sec. 5.1) by the L2
error of Eq. 28 in the displacement u and in the maximum shear stress
sigma^t = (sigma_max - sigma_min) / 2 (the radius of the largest Mohr circle,
from the principal stresses of Hooke's law, Eqs. 1 and 3).

Readings (the paper does not fix the discrete evaluation):
* fields are evaluated at the centroid of every solid voxel, one point per
  Q1 element: the strain from the element's shape-function gradients there,
  sigma = D(E_voxel, nu) eps, the displacement as the mean of the 8 corners;
* clamped and unused lattice nodes carry zero displacement;
* the integral over the solid in Eq. 28 is the midpoint rule over solid voxels
  (unit volume each) and the supremum is taken over the same points:
  E_2 = sqrt(mean_v (|chi_M - chi_S|_v / max_v |chi_S|_v)^2), with |.| the
  Euclidean norm for u and the absolute value for sigma^t.
"""
from __future__ import annotations

import numpy as np

from . import fem


def lattice_displacement(mesh, x):
    """(NZ, NY, NX, 3) displacement on every lattice node from the free-dof
    vector x (node-major dofs); clamped and unused nodes are zero."""
    U = np.zeros((mesh.NX * mesh.NY * mesh.NZ, 3))
    U[mesh.free_nodes] = np.asarray(x, dtype=float).reshape(-1, 3)
    return U.reshape(mesh.NZ, mesh.NY, mesh.NX, 3)


def voxel_fields_lattice(solid, E, nu, U):
    """Per solid voxel (in flat voxel order): the Voigt stress (xx, yy, zz, yz,
    xz, xy), the maximum shear stress and the centroid displacement, from the
    lattice displacement U (NZ, NY, NX, 3)."""
    solid = np.asarray(solid, dtype=bool)
    nz, ny, nx = solid.shape
    vox = np.flatnonzero(solid.ravel())
    k, r = np.divmod(vox, nx * ny)
    j, i = np.divmod(r, nx)
    Ue = np.empty((vox.size, 8, 3))
    for a, (cx, cy, cz) in enumerate(fem.LOCAL_NODES):
        Ue[:, a] = U[k + cz, j + cy, i + cx]
    B = fem.strain_displacement(fem.shape_gradients(0.5, 0.5, 0.5))      # 6 x 24 at the centroid
    eps = Ue.reshape(vox.size, 24) @ B.T
    D1 = fem.elasticity_matrix(1.0, nu)
    sig = (eps @ D1.T) * np.asarray(E, dtype=float).ravel()[vox][:, None]
    T = np.empty((vox.size, 3, 3))
    T[:, 0, 0], T[:, 1, 1], T[:, 2, 2] = sig[:, 0], sig[:, 1], sig[:, 2]
    T[:, 1, 2] = T[:, 2, 1] = sig[:, 3]
    T[:, 0, 2] = T[:, 2, 0] = sig[:, 4]
    T[:, 0, 1] = T[:, 1, 0] = sig[:, 5]
    w = np.linalg.eigvalsh(T)
    return sig, 0.5 * (w[:, 2] - w[:, 0]), Ue.mean(axis=1), vox


def voxel_fields(problem, mesh, x):
    """voxel_fields_lattice for a Problem's solution vector x over its free dofs."""
    return voxel_fields_lattice(problem.solid, problem.E, problem.nu, lattice_displacement(mesh, x))


def e2_error(approx, exact):
    """Eq. 28 under the midpoint reading: per-point values (n,) or vectors (n, 3)."""
    approx = np.asarray(approx, dtype=float)
    exact = np.asarray(exact, dtype=float)
    if exact.ndim == 2:
        d = np.linalg.norm(approx - exact, axis=1)
        s = np.linalg.norm(exact, axis=1).max()
    else:
        d = np.abs(approx - exact)
        s = np.abs(exact).max()
    return float(np.sqrt(np.mean((d / s) ** 2)))
