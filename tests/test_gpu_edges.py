"""Edge cases of the solver and of the method, through the C ABI.

* b = 0 gives x = 0 without iterating; an exact initial guess needs no
  iteration; a capped run reports NOT_CONVERGED with its true residual and
  can be restarted from its iterate.
* One grain holding the whole solid (no interfaces, no contact grids, no
  mortar dofs): the coarse space is the correction vector A_g^-1 b alone, so
  the first pass M_G^-1 b is the exact solution.
* Every interface node a mortar node (nu_c = N_c): Q^o is the identity and
  the first pass is again the exact solution (the paper's appendix).
Both limits are checked against a sparse direct solve.
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
def base():
    _torch()
    from oracle import fem
    from paper_2509_19777_amd import hplmm as hp
    p = synth.config_pores(12, 4, seed=3)
    A, b, mesh = fem.assemble(p)
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=2)
    S.setup()
    return p, A, b, S


def test_zero_rhs(base):
    torch = _torch()
    p, A, b, S = base
    z = torch.zeros(A.shape[0], dtype=torch.float64, device="cuda")
    x0 = torch.ones_like(z)
    x, info = S.solve(b=z, x0=x0)
    assert info["status"] == "OK" and info["iters"] == 0
    assert torch.count_nonzero(x).item() == 0


def test_exact_initial_guess(base):
    p, A, b, S = base
    x1, i1 = S.solve(rtol=1e-10, restart=50, maxit=300)
    assert i1["status"] == "OK"
    x2, i2 = S.solve(x0=x1, rtol=1e-8)
    assert i2["status"] == "OK" and i2["iters"] == 0
    assert np.array_equal(x2.cpu().numpy(), x1.cpu().numpy())


def test_capped_run_and_restart(base):
    p, A, b, S = base
    xa, ia = S.solve(rtol=1e-12, restart=50, maxit=5)
    assert ia["status"] == "NOT_CONVERGED" and ia["iters"] == 5
    true_rel = np.linalg.norm(b - A @ xa.cpu().numpy()) / np.linalg.norm(b)
    assert abs(true_rel - ia["rel_res"]) <= 1e-8 * true_rel
    xb, ib = S.solve(x0=xa, rtol=1e-8, restart=50, maxit=300)
    assert ib["status"] == "OK"
    assert np.linalg.norm(b - A @ xb.cpu().numpy()) / np.linalg.norm(b) < 1e-8


@pytest.mark.parametrize("prec", [64, 16])
def test_single_grain_first_pass_is_exact(prec):
    _torch()
    import scipy.sparse.linalg as spla
    from oracle import fem
    from paper_2509_19777_amd import hplmm as hp
    p = synth.config_pores(12, 4, seed=3)
    lab = np.where(p.solid > 0, 0, -1).astype(np.int32)
    p1 = dataclasses.replace(p, labels=lab, n_grains=1)
    A, b, mesh = fem.assemble(p1)
    sysm, part = hp.build_problem(p1)
    assert part.n_ifaces == 0 and part.n_contacts == 0
    S = hp.Solver(sysm, part, n_mortar=2, smoother_precision=prec)
    S.setup()
    sz = S.sizes()
    assert sz["n_mortar"] == 0 and sz["n_coarse"] == 1
    xs = spla.spsolve(A.tocsc(), b)
    assert _rel(S.apply(S.b, 1).cpu().numpy(), xs) <= 1e-10
    x, info = S.solve(rtol=1e-8)
    assert info["status"] == "OK" and info["iters"] <= 1
    assert np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8


def test_every_interface_node_a_mortar(base):
    import scipy.sparse.linalg as spla
    from paper_2509_19777_amd import hplmm as hp
    p, A, b, _ = base
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=10 ** 6)
    S.setup()
    N_c = np.diff(part.iface_ptr)
    nu = S.query(1, np.int32)
    assert nu.size == N_c.sum()          # every interface node carries a mortar
    xs = spla.spsolve(A.tocsc(), b)
    assert _rel(S.apply(S.b, 1).cpu().numpy(), xs) <= 1e-10
