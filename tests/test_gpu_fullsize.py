"""The 64^3 headline workload in the configuration bench.py times (n = 4,
FP64 and BF16 smoother): checks against the oracle's assembly through
properties that hold at any size.

* SpMV equals the oracle's A x (1e-14 normwise).
* Grain smoother local exactness: R_g (r - A M_g^-1 r) = 0 on every grain
  interior (Eq. 26, disjoint blocks), relative to |r|.
* M_G^-1 A is an A-projector: M_G^-1 A (M_G^-1 A v) = M_G^-1 A v (Eq. 18).
* Eq. 16 composition: M^-1 r = z1 + M_CG^-1 (r - A z1) with z1 = M_G^-1 r.
* The FGMRES solution has a true residual below 1e-8 measured with the
  oracle's matrix, and two runs are bitwise identical.

and, block by block against the oracle's own local factorisations
(oracle.hplmm.LocalSmoothers: every grain interior and contact grid of the
workload, without the dense coarse space that makes the whole oracle slow at
this size), M_zeta^-1, M_g^-1 and M_CG^-1 in both smoother forms.
"""
import numpy as np
import pytest

from paper_2509_19777_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import fem
    from paper_2509_19777_amd import hplmm as hp
    p = synth.config_grf(64, 8, seed=2, n_mortar=4)
    A, b, mesh = fem.assemble(p)
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=4)
    S.setup()
    return p, A, b, mesh, part, S


def _cu(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def test_spmv_full(big):
    p, A, b, mesh, part, S = big
    x = synth.random_vector(A.shape[0], 21)
    y = S.spmv(_cu(x)).cpu().numpy()
    assert np.linalg.norm(y - A @ x) <= 1e-14 * np.linalg.norm(A @ x)


def test_grain_smoother_exact_full(big):
    p, A, b, mesh, part, S = big
    r = synth.random_vector(A.shape[0], 22)
    z = S.apply(_cu(r), 4).cpu().numpy()
    res = r - A @ z
    grain_dofs = np.repeat(part.node_grain >= 0, 3)
    assert np.abs(res[grain_dofs]).max() <= 1e-10 * np.abs(r).max()
    assert np.all(z[~grain_dofs] == 0.0)


def test_coarse_projector_full(big):
    p, A, b, mesh, part, S = big
    v = synth.random_vector(A.shape[0], 23)
    y1 = S.apply(_cu(A @ v), 1).cpu().numpy()
    y2 = S.apply(_cu(A @ y1), 1).cpu().numpy()
    assert np.linalg.norm(y2 - y1) <= 1e-9 * np.linalg.norm(y1)


def test_multiplicative_composition_full(big):
    p, A, b, mesh, part, S = big
    r = synth.random_vector(A.shape[0], 24)
    z = S.apply(_cu(r), 0).cpu().numpy()
    z1 = S.apply(_cu(r), 1).cpu().numpy()
    z2 = S.apply(_cu(r - A @ z1), 2).cpu().numpy()
    assert np.linalg.norm(z - (z1 + z2)) <= 1e-10 * np.linalg.norm(z)


def test_solve_full(big):
    p, A, b, mesh, part, S = big
    x1, info = S.solve(rtol=1e-8, restart=50, maxit=300)
    assert info["status"] == "OK"
    xg = x1.cpu().numpy()
    assert np.linalg.norm(b - A @ xg) / np.linalg.norm(b) < 1e-8
    x2, _ = S.solve(rtol=1e-8, restart=50, maxit=300)
    assert np.array_equal(xg, x2.cpu().numpy())
    # graph replay and eager launches give the same bits
    S.use_graphs(False)
    x3, _ = S.solve(rtol=1e-8, restart=50, maxit=300)
    S.use_graphs(True)
    assert np.array_equal(xg, x3.cpu().numpy())


def test_second_setup_same_bits(big):
    """A second set-up on the same handle starts from what the first left in
    the arena: only the tiles inside each block's envelope are cleared, the
    coupling blocks are gathered on the side stream and the fronts receive
    their children's update matrices by parent tile.  Its preconditioner
    gives the first one's bits."""
    p, A, b, mesh, part, S = big
    r = np.random.default_rng(7).standard_normal(A.shape[0])
    z1 = S.apply(_cu(r), 0).cpu().numpy()
    S.setup()
    z2 = S.apply(_cu(r), 0).cpu().numpy()
    assert np.array_equal(z1, z2)


def test_solve_full_bf16_smoother(big):
    from paper_2509_19777_amd import hplmm as hp
    p, A, b, mesh, part, S = big
    S16 = hp.Solver(S.system, part, n_mortar=4, smoother_precision=16)
    S16.setup()
    x, info = S16.solve(rtol=1e-8, restart=50, maxit=300)
    assert info["status"] == "OK"
    assert np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8


def test_solve_full_fp32_inverse_smoother(big):
    # S formed in FP64 and stored in FP32 (the automatic choice at precision 32)
    from paper_2509_19777_amd import hplmm as hp
    p, A, b, mesh, part, S = big
    S32 = hp.Solver(S.system, part, n_mortar=4, smoother_precision=32)
    assert S32.smoother_form() == "inverse"
    S32.setup()
    x, info = S32.solve(rtol=1e-8, restart=50, maxit=300)
    assert info["status"] == "OK"
    assert np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8


def test_autotuned_solve_full(big):
    # the shapes the autotuner picks at full size solve to the same bar, and
    # M^-1 agrees with the default shapes to rounding
    p, A, b, mesh, part, S = big
    r = _cu(synth.random_vector(A.shape[0], 25))
    z0 = S.apply(r, 0).cpu().numpy()
    recs = S.autotune(reps=3)
    print("autotune:", [(rc["kind"], rc["index"], rc["target"], rc["waves"], round(rc["t_default_us"], 1),
                         round(rc["t_best_us"], 1)) for rc in recs])
    z1 = S.apply(r, 0).cpu().numpy()
    assert np.linalg.norm(z1 - z0) <= 1e-12 * np.linalg.norm(z0)
    x, info = S.solve(rtol=1e-8, restart=50, maxit=300)
    assert info["status"] == "OK"
    assert np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8
    S.set_tuning([])


@pytest.fixture(scope="module")
def local_oracle(big):
    # the oracle's grain and contact-grid blocks of the full workload (the
    # dense coarse space is left out: it is what makes the whole oracle slow)
    from scipy.linalg import lapack
    from oracle import hplmm as oh
    p, A, b, mesh, part, S = big
    L = oh.LocalSmoothers(p, A, mesh)
    kappa = 0.0
    for d, ch in zip(L.grain_dofs + L.contact_dofs, L.grain_chol + L.contact_chol):
        if ch is None:
            continue
        anorm = np.abs(A[d][:, d]).sum(axis=0).max()
        rcond, info = lapack.dpocon(ch[0], anorm, uplo='L')
        kappa = max(kappa, 1.0 / rcond)
    print(f"64^3: {len(L.grain_dofs)} grains, {len(L.contact_dofs)} contact grids, max kappa_1 {kappa:.3e}")
    return L, kappa


@pytest.fixture(scope="module")
def factors_solver(big):
    from paper_2509_19777_amd import hplmm as hp
    p, A, b, mesh, part, S = big
    Sf = hp.Solver(S.system, part, n_mortar=4, smoother_form="factors")
    Sf.setup()
    return Sf


@pytest.mark.parametrize("which", [3, 4, 2])
@pytest.mark.parametrize("form", ["inverse", "factors"])
def test_local_smoothers_full_vs_oracle(big, local_oracle, factors_solver, which, form):
    # M_zeta^-1, M_g^-1 and M_CG^-1 at full size against per-block dense
    # Cholesky solves (Eqs. 25-26): normwise within max(1e-12, 10 kappa u)
    # (kappa_1 of the worst block, an upper estimate of kappa_2) and within the
    # fixed 1e-12; every entry within 1e-11 of the largest
    p, A, b, mesh, part, S = big
    L, kappa = local_oracle
    if form == "factors":
        S = factors_solver
    op = {3: L.apply_Mzeta, 4: L.apply_Mg, 2: L.apply_MCG}[which]
    bar = max(1e-12, 10.0 * kappa * 2.0 ** -53)
    r = synth.random_vector(A.shape[0], 26 + which)
    zo = op(r)
    z = S.apply(_cu(r), which).cpu().numpy()
    nrm = np.linalg.norm(z - zo) / np.linalg.norm(zo)
    ele = np.abs(z - zo).max() / np.abs(zo).max()
    print(f"64^3 which {which} ({form}): normwise {nrm:.2e} (bar {bar:.1e}), elementwise {ele:.2e}")
    assert nrm <= bar and nrm <= 1e-12
    assert ele <= 1e-11
