"""Pins of the stress-recovery oracle and the Eq. 28 metric against closed
forms: linear displacement fields (constant strain), principal values of
Hooke's law, rotation invariance of the Mohr radius, and the metric's
scaling."""
import numpy as np

from oracle import fem, stress
from paper_2509_19777_amd import synth


def _linear_field(shape, G, t):
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    X = np.stack([i, j, k], axis=-1).astype(float)
    return X @ np.asarray(G, dtype=float).T + np.asarray(t, dtype=float)


def _rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q @ np.diag(np.sign(np.diag(r)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def _solid():
    p = synth.config_pores(8, 4, seed=3)
    return p.solid, p.E, p.nu


def test_linear_field_gives_hooke_stress_everywhere():
    solid, E, nu = _solid()
    G = np.random.default_rng(1).standard_normal((3, 3))
    U = _linear_field(solid.shape, G, [0.3, -0.2, 0.5])
    sig, st, ucen, vox = stress.voxel_fields_lattice(solid, E, nu, U)
    eps = 0.5 * (G + G.T)
    lam, mu = fem.lame(1.0, nu)
    S1 = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps        # stress per unit E
    Ev = E.ravel()[vox]
    want = np.stack([S1[0, 0], S1[1, 1], S1[2, 2], S1[1, 2], S1[0, 2], S1[0, 1]])
    assert np.allclose(sig, Ev[:, None] * want[None, :], rtol=1e-13, atol=1e-13)
    # the centroid displacement of a linear field is the field at the centroid
    k, r = np.divmod(vox, solid.shape[1] * solid.shape[2])
    j, i = np.divmod(r, solid.shape[2])
    C = np.stack([i + 0.5, j + 0.5, k + 0.5], axis=1)
    assert np.allclose(ucen, C @ G.T + [0.3, -0.2, 0.5], rtol=1e-14, atol=1e-13)


def test_principal_strains_give_mohr_radius():
    # eps = R diag(g) R^T: principal stresses lam tr + 2 mu g_i, radius mu (g_max - g_min)
    solid, E, nu = _solid()
    lam, mu = fem.lame(1.0, nu)
    g = np.array([0.7, -0.4, 0.1])
    for seed in (0, 5):
        R = _rotation(seed)
        G = R @ np.diag(g) @ R.T
        _, st, _, vox = stress.voxel_fields_lattice(solid, E, nu, _linear_field(solid.shape, G, [0, 0, 0]))
        assert np.allclose(st, E.ravel()[vox] * mu * (g.max() - g.min()), rtol=1e-12)


def test_pure_shear_and_hydrostatic():
    solid, E, nu = _solid()
    lam, mu = fem.lame(1.0, nu)
    gam = 0.02
    G = np.zeros((3, 3))
    G[0, 1] = gam                        # u_x = gam * y: engineering shear gam, tensor shear gam / 2
    _, st, _, vox = stress.voxel_fields_lattice(solid, E, nu, _linear_field(solid.shape, G, [0, 0, 0]))
    assert np.allclose(st, E.ravel()[vox] * mu * gam, rtol=1e-12)
    _, st0, _, _ = stress.voxel_fields_lattice(solid, E, nu, _linear_field(solid.shape, 0.01 * np.eye(3), [1, 2, 3]))
    assert np.abs(st0).max() <= 1e-15


def test_rigid_motion_is_stress_free():
    solid, E, nu = _solid()
    W = np.array([[0, -0.3, 0.2], [0.3, 0, -0.1], [-0.2, 0.1, 0]])    # linearised rotation
    sig, st, _, _ = stress.voxel_fields_lattice(solid, E, nu, _linear_field(solid.shape, W, [1, -1, 2]))
    assert np.abs(sig).max() <= 1e-14 and np.abs(st).max() <= 1e-14


def test_free_dof_vector_puts_zero_on_clamped_nodes():
    p = synth.config_pores(8, 4, seed=3)
    A, b, mesh = fem.assemble(p)
    # u = (0, 0, c z): vanishes on the clamped plane, so the free-dof vector
    # carries the whole linear field
    c = 0.01
    x = np.zeros(3 * mesh.n)
    x[2::3] = c * mesh.xyz[:, 2]
    sig, st, ucen, vox = stress.voxel_fields(p, mesh, x)
    lam, mu = fem.lame(1.0, p.nu)
    Ev = p.E.ravel()[vox]
    assert np.allclose(sig[:, 2], Ev * (lam + 2 * mu) * c, rtol=1e-12)
    assert np.allclose(sig[:, 0], Ev * lam * c, rtol=1e-12)
    assert np.allclose(ucen[:, 2], c * (vox // 64 + 0.5), rtol=1e-12)


def test_e2_metric_closed_forms():
    rng = np.random.default_rng(2)
    s = rng.standard_normal(500)
    u = rng.standard_normal((500, 3))
    assert stress.e2_error(s, s) == 0.0
    # approx = 0: sqrt(mean chi^2) / sup |chi|
    assert np.isclose(stress.e2_error(np.zeros(500), s), np.sqrt(np.mean(s ** 2)) / np.abs(s).max(), rtol=1e-14)
    un = np.linalg.norm(u, axis=1)
    assert np.isclose(stress.e2_error(1.1 * u, u), 0.1 * np.sqrt(np.mean(un ** 2)) / un.max(), rtol=1e-12)
    # a single point off by delta: delta / (sup * sqrt(n))
    a = s.copy()
    a[7] += 0.25
    assert np.isclose(stress.e2_error(a, s), 0.25 / np.abs(s).max() / np.sqrt(500), rtol=1e-12)
