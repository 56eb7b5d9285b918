"""Oracle: Q1 (trilinear hexahedral) Galerkin FEM for small-strain isotropic
linear elasticity on a voxel grid.  TEST INFRASTRUCTURE ONLY.

Follows Sec. 2 of the paper: the momentum balance and Hooke's law (Eq. 1),
Dirichlet/Neumann boundary conditions (Eq. 2), the isotropic stiffness tensor
in Lame form (Eq. 3) and the Galerkin discretisation on a Cartesian grid with
trilinear shape functions, which yields the symmetric system A x = b (Eq. 4).

Readings (the paper does not fix these for our synthetic workloads):
* voxel edge h = 1; one Q1 element per solid voxel;
* nodes on the plane z = 0 are clamped and eliminated from the system;
* a uniform traction t acts on the top face z = nz of every solid voxel of the
  top layer, distributed as the consistent Q1 load t/4 per face node;
* free nodes are the remaining nodes touched by a solid voxel, numbered in
  ascending lattice order (x fastest); dofs are node-major: 3*node + comp.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def lame(E, nu):
    """Lame parameters of Eq. (3) from Young's modulus and Poisson's ratio."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def elasticity_matrix(E, nu):
    """6x6 Voigt matrix of Eq. (3) (order xx, yy, zz, yz, xz, xy; engineering
    shear strains), i.e. C_ijkl = lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk)."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


LOCAL_NODES = np.array([(a & 1, (a >> 1) & 1, (a >> 2) & 1) for a in range(8)])


def shape_gradients(xi, eta, zeta):
    """Gradients of the 8 trilinear shape functions on the unit cube at one
    point; local node a sits at corner (a&1, a>>1&1, a>>2&1)."""
    p = np.array([xi, eta, zeta])
    G = np.zeros((8, 3))
    for a, c in enumerate(LOCAL_NODES):
        f = [p[d] if c[d] else 1.0 - p[d] for d in range(3)]
        s = [1.0 if c[d] else -1.0 for d in range(3)]
        G[a, 0] = s[0] * f[1] * f[2]
        G[a, 1] = f[0] * s[1] * f[2]
        G[a, 2] = f[0] * f[1] * s[2]
    return G


def strain_displacement(G):
    """6x24 matrix B mapping the element dofs (3*a + comp) to Voigt strain."""
    B = np.zeros((6, 24))
    for a in range(8):
        gx, gy, gz = G[a]
        c = 3 * a
        B[0, c + 0] = gx
        B[1, c + 1] = gy
        B[2, c + 2] = gz
        B[3, c + 1] = gz
        B[3, c + 2] = gy
        B[4, c + 0] = gz
        B[4, c + 2] = gx
        B[5, c + 0] = gy
        B[5, c + 1] = gx
    return B


def element_stiffness(E=1.0, nu=0.3, order=2):
    """K_e = int_{[0,1]^3} B^T D B dV by tensor Gauss-Legendre quadrature.
    Two points per direction integrate the (bi-quadratic) integrand exactly."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    xg = 0.5 * (xg + 1.0)
    wg = 0.5 * wg
    D = elasticity_matrix(E, nu)
    K = np.zeros((24, 24))
    for i, wi in zip(xg, wg):
        for j, wj in zip(xg, wg):
            for k, wk in zip(xg, wg):
                B = strain_displacement(shape_gradients(i, j, k))
                K += wi * wj * wk * (B.T @ D @ B)
    # the exact integral is symmetric; remove the rounding asymmetry of B^T D B
    return 0.5 * (K + K.T)


class Mesh:
    """Node bookkeeping of a voxel solid.

    free_nodes: lattice ids of the free nodes (ascending);
    lat2free:   lattice id -> free index, or -1;
    xyz:        (n_free, 3) integer lattice coordinates of free nodes.
    """

    def __init__(self, solid):
        solid = np.asarray(solid, dtype=bool)
        nz, ny, nx = solid.shape
        self.nx, self.ny, self.nz = nx, ny, nz
        self.NX, self.NY, self.NZ = nx + 1, ny + 1, nz + 1
        touched = np.zeros((nz + 1, ny + 1, nx + 1), dtype=bool)
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    touched[dz:dz + nz, dy:dy + ny, dx:dx + nx] |= solid
        touched[0] = False  # clamped plane z = 0
        self.free_nodes = np.flatnonzero(touched.ravel())
        self.lat2free = -np.ones(touched.size, dtype=np.int64)
        self.lat2free[self.free_nodes] = np.arange(self.free_nodes.size)
        k, r = np.divmod(self.free_nodes, self.NX * self.NY)
        j, i = np.divmod(r, self.NX)
        self.xyz = np.stack([i, j, k], axis=1).astype(np.int64)
        self.n = self.free_nodes.size
        self.solid = solid

    def lattice_id(self, i, j, k):
        return i + self.NX * (j + self.NY * k)

    def voxel_nodes(self):
        """(n_solid, 8) lattice ids of the corners of every solid voxel, in the
        element's local node order, plus the voxel flat indices."""
        vox = np.flatnonzero(self.solid.ravel())
        k, r = np.divmod(vox, self.nx * self.ny)
        j, i = np.divmod(r, self.nx)
        nodes = np.empty((vox.size, 8), dtype=np.int64)
        for a, (cx, cy, cz) in enumerate(LOCAL_NODES):
            nodes[:, a] = self.lattice_id(i + cx, j + cy, k + cz)
        return nodes, vox


def assemble(problem):
    """Assemble A (scipy CSR over free dofs), b and the Mesh of a Problem.

    A = sum_e E_e * P_e^T K_hat(nu) P_e restricted to free dofs (Eq. 4);
    b = consistent top-face traction load.
    """
    mesh = Mesh(problem.solid)
    Kh = element_stiffness(1.0, problem.nu)
    nodes, vox = mesh.voxel_nodes()
    Ev = problem.E.ravel()[vox]
    fidx = mesh.lat2free[nodes]                       # (ne, 8), -1 = clamped
    dof = (3 * fidx[:, :, None] + np.arange(3)).reshape(-1, 24)
    dof[np.repeat(fidx, 3, axis=1).reshape(-1, 24) < 0] = -1
    rows = np.repeat(dof, 24, axis=1).ravel()
    cols = np.tile(dof, (1, 24)).ravel()
    vals = (Ev[:, None, None] * Kh[None, :, :]).ravel()
    keep = (rows >= 0) & (cols >= 0)
    n = 3 * mesh.n
    A = sp.coo_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    b = np.zeros(n)
    t = np.asarray(problem.traction, dtype=float)
    top = np.flatnonzero(problem.solid[-1].ravel())
    if top.size:
        j, i = np.divmod(top, mesh.nx)
        kk = mesh.nz
        for cx in (0, 1):
            for cy in (0, 1):
                f = mesh.lat2free[mesh.lattice_id(i + cx, j + cy, kk)]
                for c in range(3):
                    np.add.at(b, 3 * f + c, 0.25 * t[c])
    return A, b, mesh


def rigid_modes(xyz):
    """The six rigid-body modes (3 translations, 3 linearised rotations) on
    nodes with coordinates xyz, node-major."""
    n = xyz.shape[0]
    x, y, z = (xyz[:, d].astype(float) for d in range(3))
    R = np.zeros((3 * n, 6))
    for c in range(3):
        R[c::3, c] = 1.0
    R[0::3, 3], R[1::3, 3] = -y, x          # rotation about z
    R[1::3, 4], R[2::3, 4] = -z, y          # rotation about x
    R[0::3, 5], R[2::3, 5] = z, -x          # rotation about y
    return R


def assemble_unconstrained(solid, E, nu):
    """A over every node touched by a solid voxel, with no clamping (for the
    rigid-mode and patch tests).  Returns (A, xyz, lattice ids)."""
    solid = np.asarray(solid, dtype=bool)
    nz, ny, nx = solid.shape
    NX, NY = nx + 1, ny + 1
    vox = np.flatnonzero(solid.ravel())
    k, r = np.divmod(vox, nx * ny)
    j, i = np.divmod(r, nx)
    nodes = np.empty((vox.size, 8), dtype=np.int64)
    for a, (cx, cy, cz) in enumerate(LOCAL_NODES):
        nodes[:, a] = (i + cx) + NX * ((j + cy) + NY * (k + cz))
    used = np.unique(nodes)
    remap = -np.ones((nx + 1) * (ny + 1) * (nz + 1), dtype=np.int64)
    remap[used] = np.arange(used.size)
    Kh = element_stiffness(1.0, nu)
    Ev = np.asarray(E, dtype=float).ravel()[vox]
    f = remap[nodes]
    dof = (3 * f[:, :, None] + np.arange(3)).reshape(-1, 24)
    rows = np.repeat(dof, 24, axis=1).ravel()
    cols = np.tile(dof, (1, 24)).ravel()
    vals = (Ev[:, None, None] * Kh[None]).ravel()
    n = 3 * used.size
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    kk, rr = np.divmod(used, NX * NY)
    jj, ii = np.divmod(rr, NX)
    return A, np.stack([ii, jj, kk], axis=1), used
