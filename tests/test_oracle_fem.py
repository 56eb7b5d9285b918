"""Pins of the oracle's Q1 elasticity discretisation (paper Sec. 2, Eqs. 1-4)
against closed forms, the rigid-body null space, the patch test and the
uniaxial bar."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem
from paper_2509_19777_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_element_entries_match_hand_integration():
    g = json.load(open(os.path.join(GOLD, "q1_element_unit_cube.json")))
    K = fem.element_stiffness(g["E"], g["nu"])
    for e in g["entries"]:
        assert K[e["row"], e["col"]] == pytest.approx(e["value"], rel=1e-14)


def test_element_symmetric_psd_six_rigid_modes():
    K = fem.element_stiffness(2.5, 0.27)
    assert np.allclose(K, K.T, atol=0, rtol=0)
    w = np.linalg.eigvalsh(K)
    tol = 1e-12 * w.max()
    assert np.sum(np.abs(w) < tol) == 6
    assert np.all(w > -tol)
    R = fem.rigid_modes(fem.LOCAL_NODES)
    assert np.abs(K @ R).max() < 1e-13 * np.abs(K).max()


def test_element_quadrature_is_exact():
    # the integrand is at most quadratic per direction: 2 and 4 Gauss points agree
    assert np.allclose(fem.element_stiffness(1.0, 0.3, order=2),
                       fem.element_stiffness(1.0, 0.3, order=4), rtol=0, atol=1e-14)


def test_element_scales_linearly_in_E():
    K3, K1 = fem.element_stiffness(3.0, 0.3), fem.element_stiffness(1.0, 0.3)
    assert np.abs(K3 - 3.0 * K1).max() <= 1e-14 * np.abs(K3).max()


def test_global_unconstrained_null_space():
    p = synth.config_pores(8, 4, seed=3)
    E = np.where(p.solid > 0, np.exp(np.random.default_rng(0).standard_normal(p.solid.shape)), 0)
    A, xyz, _ = fem.assemble_unconstrained(p.solid, E, 0.3)
    R = fem.rigid_modes(xyz)
    nA = spla.norm(A, 1)
    for c in range(6):
        r = R[:, c]
        assert np.linalg.norm(A @ r) <= 1e-14 * nA * np.linalg.norm(r)


def _block(n):
    return np.ones((n, n, n), dtype=np.uint8)


def test_patch_test_linear_field_exact():
    """A general affine displacement imposed on the boundary of a pore-free
    block is reproduced exactly at the interior nodes."""
    n = 4
    solid = _block(n)
    A, xyz, _ = fem.assemble_unconstrained(solid, np.ones(solid.shape) * 1.7, 0.3)
    G = np.array([[0.01, 0.02, -0.005], [0.004, -0.03, 0.01], [0.02, 0.0, 0.015]])
    u = (xyz.astype(float) @ G.T + np.array([0.1, -0.2, 0.3])).ravel()
    bnd = np.any((xyz == 0) | (xyz == n), axis=1)
    bd = np.repeat(bnd, 3)
    Aii = A[~bd][:, ~bd].tocsc()
    Aib = A[~bd][:, bd]
    ui = spla.spsolve(Aii, -Aib @ u[bd])
    assert np.abs(ui - u[~bd]).max() < 1e-13


def test_uniaxial_bar_closed_form():
    """Roller supports on x=0, y=0, z=0 and a uniform pressure p on the top:
    u_z = -p z / E, u_x = nu p x / E, u_y = nu p y / E exactly."""
    nx, ny, nz = 3, 2, 4
    E, nu, p = 2.0, 0.3, 0.5
    solid = np.ones((nz, ny, nx), dtype=np.uint8)
    A, xyz, _ = fem.assemble_unconstrained(solid, np.full(solid.shape, E), nu)
    nn = xyz.shape[0]
    b = np.zeros(3 * nn)
    # consistent load of a uniform pressure: a quarter of each unit face per node
    for i in range(nx):
        for j in range(ny):
            for cx in (0, 1):
                for cy in (0, 1):
                    v = np.flatnonzero((xyz[:, 0] == i + cx) & (xyz[:, 1] == j + cy) & (xyz[:, 2] == nz))[0]
                    b[3 * v + 2] -= 0.25 * p
    fixed = np.zeros(3 * nn, dtype=bool)
    fixed[0::3] = xyz[:, 0] == 0
    fixed[1::3] = xyz[:, 1] == 0
    fixed[2::3] = xyz[:, 2] == 0
    free = ~fixed
    u = np.zeros(3 * nn)
    u[free] = spla.spsolve(A[free][:, free].tocsc(), b[free])
    x, y, z = (xyz[:, d].astype(float) for d in range(3))
    assert np.allclose(u[2::3], -p * z / E, atol=1e-13)
    assert np.allclose(u[0::3], nu * p * x / E, atol=1e-13)
    assert np.allclose(u[1::3], nu * p * y / E, atol=1e-13)


def test_clamped_system_symmetric_spd_and_load():
    p = synth.config_pores(8, 4, seed=5)
    A, b, mesh = fem.assemble(p)
    assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
    assert np.all(mesh.xyz[:, 2] > 0)
    # total force equals traction times the solid top area
    assert b[2::3].sum() == pytest.approx(-1.0 * p.solid[-1].sum(), rel=1e-14)
    assert np.all(b[0::3] == 0) and np.all(b[1::3] == 0)
    L = np.linalg.cholesky(A.toarray())
    assert np.all(np.isfinite(L))


def test_constrained_dofs_identity_rows():
    """oracle.constraints on the uniaxial bar: roller supports on x = 0, y = 0
    and z = 0 as identity rows reproduce the closed form exactly, and on a
    porous block the constrained system's solution is zero at the fixed dofs
    and equals the reduced system's elsewhere."""
    from oracle import constraints
    nx, ny, nz = 3, 2, 4
    E, nu, p = 2.0, 0.3, 0.5
    solid = np.ones((nz, ny, nx), dtype=np.uint8)
    A, xyz, _ = fem.assemble_unconstrained(solid, np.full(solid.shape, E), nu)
    nn = xyz.shape[0]
    b = np.zeros(3 * nn)
    for i in range(nx):
        for j in range(ny):
            for cx in (0, 1):
                for cy in (0, 1):
                    v = np.flatnonzero((xyz[:, 0] == i + cx) & (xyz[:, 1] == j + cy) & (xyz[:, 2] == nz))[0]
                    b[3 * v + 2] -= 0.25 * p
    fixed = np.zeros(3 * nn, dtype=bool)
    fixed[0::3] = xyz[:, 0] == 0
    fixed[1::3] = xyz[:, 1] == 0
    fixed[2::3] = xyz[:, 2] == 0
    Ac, bc = constraints.constrain(A, b, fixed)
    assert abs(Ac - Ac.T).max() <= 1e-15 * abs(A).max()
    u = spla.spsolve(Ac.tocsc(), bc)
    x, y, z = (xyz[:, d].astype(float) for d in range(3))
    assert np.allclose(u[2::3], -p * z / E, atol=1e-13)
    assert np.allclose(u[0::3], nu * p * x / E, atol=1e-13)
    assert np.allclose(u[1::3], nu * p * y / E, atol=1e-13)
    # porous block with the clamp eliminated and rollers on x = 0, y = 0
    pr = synth.config_pores(8, 4, seed=11, porosity=0.2)
    A2, b2, mesh = fem.assemble(pr)
    xyz2 = mesh.xyz
    f2 = np.zeros(A2.shape[0], dtype=bool)
    f2[0::3] = xyz2[:, 0] == 0
    f2[1::3] = xyz2[:, 1] == 0
    A2c, b2c = constraints.constrain(A2, b2, f2)
    u2 = spla.spsolve(A2c.tocsc(), b2c)
    assert np.all(u2[f2] == 0.0)
    free = ~f2
    ur = spla.spsolve(A2[free][:, free].tocsc(), b2[free])
    assert np.abs(u2[free] - ur).max() <= 1e-12 * np.abs(ur).max()
