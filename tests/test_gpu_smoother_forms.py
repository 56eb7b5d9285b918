"""The two forms of the smoother's local solves, through the C ABI.

The factor form applies y = W^T (W x) with W = L^-1 (two passes over the
lower tiles); the inverse form applies y = S x with S = W^T W formed in the
set-up, reading each lower tile of S once for S_ij x_j and S_ij^T x_i.  Both
are the same operator A_g^-1 / A_zeta^-1 (Eqs. 25-26) up to rounding, so each
is held to the oracle at the parity bar (1e-12 normwise) and the two to each
other at 1e-13; FGMRES takes the same number of iterations with either.
"""
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


@pytest.fixture(scope="module", params=[(16, 2), (20, 4)])
def pair(request):
    _torch()
    from oracle import fem, hplmm as oh
    from paper_2509_19777_amd import hplmm as hp
    L, n = request.param
    p = synth.config_pores(L, 4, seed=1)
    A, b, mesh = fem.assemble(p)
    H = oh.HPLMM(p, A=A, b=b, mesh=mesh, n=n)
    sysm, part = hp.build_problem(p)
    F = hp.Solver(sysm, part, n_mortar=n, smoother_form="factors")
    F.setup()
    I = hp.Solver(sysm, part, n_mortar=n, smoother_form="inverse")
    I.setup()
    return p, A, b, H, F, I


def test_forms_in_use(pair):
    p, A, b, H, F, I = pair
    assert F.smoother_form() == "factors" and I.smoother_form() == "inverse"


@pytest.mark.parametrize("which", [4, 3, 2, 0])
def test_both_forms_match_the_oracle_and_each_other(pair, which):
    p, A, b, H, F, I = pair
    ops = {0: H.apply, 2: H.apply_MCG, 3: H.apply_Mzeta, 4: H.apply_Mg}
    for seed in (5, 6):
        r = synth.random_vector(A.shape[0], seed)
        zf = F.apply(_cu(r), which).cpu().numpy()
        zi = I.apply(_cu(r), which).cpu().numpy()
        zo = ops[which](r)
        assert _rel(zf, zo) <= 1e-12 and _rel(zi, zo) <= 1e-12, (which, _rel(zf, zo), _rel(zi, zo))
        assert _rel(zi, zf) <= 1e-13, (which, _rel(zi, zf))


def test_inverse_form_is_deterministic(pair):
    p, A, b, H, F, I = pair
    r = _cu(synth.random_vector(A.shape[0], 7))
    z1 = I.apply(r, 0).cpu().numpy()
    z2 = I.apply(r, 0).cpu().numpy()
    assert np.array_equal(z1, z2)


def test_same_iterations(pair):
    p, A, b, H, F, I = pair
    xf, inf_ = F.solve(rtol=1e-8, restart=50, maxit=300)
    xi, ini = I.solve(rtol=1e-8, restart=50, maxit=300)
    assert inf_["status"] == ini["status"] == "OK"
    assert inf_["iters"] == ini["iters"]
    assert np.linalg.norm(b - A @ xi.cpu().numpy()) / np.linalg.norm(b) < 1e-8


def test_profiler_sees_one_pass_and_the_sums(pair):
    p, A, b, H, F, I = pair
    torch = _torch()
    r = _cu(synth.random_vector(A.shape[0], 8))
    for S, smoother_launches, sums in ((F, 4, (0,)), (I, 2, (1, 2))):
        S.profile(["gemv_smoother", "smoother_reduce"])
        S.apply(r, 0)
        torch.cuda.synchronize()
        res = S.profile_results()
        S.profile([])
        assert res["gemv_smoother"]["launches"] == smoother_launches
        # one sum launch per dense set with a matrix of more than one tile row
        assert res["smoother_reduce"]["launches"] in sums
    # the inverse form reads the smoother's tiles once: about half the bytes
    fb, ib = F.algorithmic_bytes()["apply"], I.algorithmic_bytes()["apply"]
    assert ib < fb


def test_auto_form_by_precision():
    # the inverse form at every precision: at reduced precision its S is the
    # Gram matrix of the rounded inverse factor, positive definite however
    # coarse the rounding
    _torch()
    from paper_2509_19777_amd import hplmm as hp
    p = synth.config_pores(12, 4, seed=3)
    sysm, part = hp.build_problem(p)
    for prec, form in ((64, "inverse"), (32, "inverse"), (16, "inverse")):
        assert hp.Solver(sysm, part, n_mortar=2, smoother_precision=prec).smoother_form() == form
