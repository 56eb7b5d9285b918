"""The matrix-free fine operator (hplmm_set_voxel_operator) against the
oracle's assembled matrix and against the library's assembled SpMV.

Tolerances: products 1e-14 normwise (the same element sums in another
order).  The matrix-free operator is A + F with |F| <= 8u |A| entrywise (at
most eight element terms per entry, summed in another order); the
preconditioner feeds A z through the local inverses A_i^-1 twice (contact,
then grain smoother), so an application may move by up to about
2 * 8u * kappa_max relative, kappa_max the largest local condition number
(from the oracle): applications are held to 1e-12 + 16 u kappa_max.  FGMRES
iterations within one of the oracle's.
"""
import dataclasses

import numpy as np
import pytest

from paper_2509_19777_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _cu(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def case():
    _torch()
    from oracle import fem, hplmm as oh
    from paper_2509_19777_amd import hplmm as hp
    p = synth.config_grf(16, 8, seed=2, n_mortar=4)
    A, b, mesh = fem.assemble(p)
    H = oh.HPLMM(p, A=A, b=b, mesh=mesh, n=4)
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=4)
    S.setup()
    return p, A, b, H, S


def test_products_match(case):
    p, A, b, H, S = case
    x = synth.random_vector(A.shape[0], 5)
    y_asm = S.spmv(_cu(x)).cpu().numpy()
    S.set_voxel_operator(p)
    y_mf = S.spmv(_cu(x)).cpu().numpy()
    assert _rel(y_mf, A @ x) <= 1e-14
    assert _rel(y_mf, y_asm) <= 1e-14
    S.set_voxel_operator(None)
    assert np.array_equal(S.spmv(_cu(x)).cpu().numpy(), y_asm)


def test_preconditioner_and_solve(case):
    from oracle import gmres
    p, A, b, H, S = case
    S.set_voxel_operator(p)
    r = synth.random_vector(A.shape[0], 9)
    kappa = H.max_local_condition()
    bar = 1e-12 + 16 * np.finfo(float).eps / 2 * kappa
    assert _rel(S.apply(_cu(r), 0).cpu().numpy(), H.apply(r)) <= bar, (kappa, bar)
    ro = gmres.gmres(A, b, H.apply, tol=1e-8, restart=50, flexible=True)
    x, info = S.solve(rtol=1e-8, restart=50, maxit=300)
    assert info["status"] == "OK" and abs(info["iters"] - ro.iters) <= 1
    assert np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8
    # captured graphs follow the operator: eager and graph replays agree
    S.use_graphs(False)
    xe, ie = S.solve(rtol=1e-8, restart=50, maxit=300)
    S.use_graphs(True)
    for _ in range(2):
        xg, ig = S.solve(rtol=1e-8, restart=50, maxit=300)
        assert ig["iters"] == ie["iters"] and np.array_equal(xg.cpu().numpy(), xe.cpu().numpy())
    S.set_voxel_operator(None)


def test_mismatched_grid_is_refused(case):
    from paper_2509_19777_amd import hplmm as hp
    p, A, b, H, S = case
    x = _cu(synth.random_vector(A.shape[0], 6))
    y0 = S.spmv(x).cpu().numpy()
    for bad in (dataclasses.replace(p, nu=0.25), dataclasses.replace(p, E=p.E * 1.001),
                dataclasses.replace(p, solid=p.solid[:-1], E=p.E[:-1])):
        with pytest.raises(hp.HplmmError):
            S.set_voxel_operator(bad)
        assert np.array_equal(S.spmv(x).cpu().numpy(), y0)   # still the assembled operator


def test_full_size_solve():
    _torch()
    from oracle import fem
    from paper_2509_19777_amd import hplmm as hp
    p = synth.config_grf(64, 8, seed=2, n_mortar=4)
    A, b, mesh = fem.assemble(p)
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=4)
    S.set_voxel_operator(p)
    S.setup()
    x = synth.random_vector(A.shape[0], 21)
    assert _rel(S.spmv(_cu(x)).cpu().numpy(), A @ x) <= 1e-14
    xs, info = S.solve(rtol=1e-8, restart=50, maxit=300)
    assert info["status"] == "OK"
    assert np.linalg.norm(b - A @ xs.cpu().numpy()) / np.linalg.norm(b) < 1e-8
