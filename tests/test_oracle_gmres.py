"""Pins of the oracle's Krylov solver (paper Sec. 5, reading R10)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem, gmres, hplmm
from paper_2509_19777_amd import synth


def test_gmres_exact_in_n_steps_dense():
    """Without restart GMRES is exact after n steps (Krylov space = R^n)."""
    rng = np.random.default_rng(0)
    n = 12
    M = rng.standard_normal((n, n)) + n * np.eye(n)
    A = sp.csr_matrix(M)
    b = rng.standard_normal(n)
    r = gmres.gmres(A, b, lambda v: v, tol=1e-30, restart=n, maxit=n)
    assert np.linalg.norm(r.x - np.linalg.solve(M, b)) < 1e-12 * np.linalg.norm(b)


def test_gmres_minimises_residual_over_krylov_space():
    """After k steps the residual equals the least-squares minimum over
    x0 + M^-1 K_k(A M^-1, r0), computed by brute force."""
    rng = np.random.default_rng(1)
    n, k = 30, 6
    M = rng.standard_normal((n, n)) + 4 * np.eye(n)
    D = np.diag(1.0 + rng.random(n))
    A = sp.csr_matrix(M)
    b = rng.standard_normal(n)
    prec = lambda v: D @ v
    r = gmres.gmres(A, b, prec, tol=0, restart=50, maxit=k, max_steps=k)
    Kr = np.zeros((n, k))
    v = b.copy()
    for j in range(k):
        Kr[:, j] = v
        v = M @ (D @ v)
    Y = D @ Kr
    c, *_ = np.linalg.lstsq(M @ Y, b, rcond=None)
    best = np.linalg.norm(b - M @ (Y @ c))
    assert np.linalg.norm(b - A @ r.x) == pytest.approx(best, rel=1e-8)


def test_flexible_equals_standard_for_fixed_M():
    p = synth.config_pores(12, 4, seed=7)
    A, b, mesh = fem.assemble(p)
    H = hplmm.HPLMM(p, A=A, b=b, mesh=mesh, n=2)
    r1 = gmres.gmres(A, b, H.apply, tol=1e-8)
    r2 = gmres.gmres(A, b, H.apply, tol=1e-8, flexible=True)
    assert r1.converged and r2.converged
    assert abs(r1.iters - r2.iters) <= 1
    assert np.linalg.norm(r1.x - r2.x) <= 1e-7 * np.linalg.norm(r1.x)


@pytest.mark.slow
def test_hplmm_gmres_solves_pore_cube():
    """16^3 pore cube: GMRES with M converges to a true residual below 1e-8,
    agrees with a sparse direct solve, and needs no more iterations as n grows
    (soft check of the paper's observation (1) in Sec. 6.2)."""
    p = synth.config_pores(16, 4, seed=1)
    A, b, mesh = fem.assemble(p)
    xs = spla.spsolve(A.tocsc(), b)
    its = []
    for n in (1, 2, 4):
        H = hplmm.HPLMM(p, A=A, b=b, mesh=mesh, n=n)
        r = gmres.gmres(A, b, H.apply, tol=1e-8, flexible=True)
        assert r.converged and r.rel_res < 1e-8
        assert np.linalg.norm(r.x - xs) <= 1e-6 * np.linalg.norm(xs)
        its.append(r.iters)
    assert its[0] >= its[1] >= its[2]
