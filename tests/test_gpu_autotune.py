"""Launch-shape autotuning of the solve phase, through the C ABI.

Every shape the autotuner can pick computes the same M^-1 up to the order of
the partial sums, so each is held to the oracle at the preconditioner bar
(1e-12 normwise); a pinned set of shapes reproduces its results bit for bit;
captured solver graphs follow a change of shapes.
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


def _set_launches(S):
    # smoother and basis GEMV launches: grain W, W^T, contact W, W^T, X^T, X
    # (factor form) or grain S, contact S, X^T, X (inverse form)
    return 4 if S.smoother_form() == "inverse" else 6


@pytest.fixture(scope="module")
def case():
    _torch()
    from oracle import fem, hplmm as oh
    from paper_2509_19777_amd import hplmm as hp
    p = synth.config_pores(16, 4, seed=1)
    A, b, mesh = fem.assemble(p)
    H = oh.HPLMM(p, A=A, b=b, mesh=mesh, n=4)
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=4)
    S.setup()
    return p, A, b, H, S, (sysm, part)


def test_autotune_records_and_parity(case):
    p, A, b, H, S, _ = case
    r = synth.random_vector(A.shape[0], 10)
    z0 = S.apply(_cu(r), 0).cpu().numpy()
    recs = S.autotune(reps=3)
    assert recs, "no launch was tuned"
    kinds = {rc["kind"] for rc in recs}
    assert kinds >= {0, 1, 2}
    for rc in recs:
        assert rc["waves"] in (4, 16)
        assert rc["t_best_us"] <= rc["t_default_us"] + 1e-9
        assert rc["t_default_us"] > 0
    assert S.tuning() == recs
    z1 = S.apply(_cu(r), 0).cpu().numpy()
    assert _rel(z1, H.apply(r)) <= 1e-12
    assert _rel(z1, z0) <= 1e-12
    x, info = S.solve(rtol=1e-8, restart=50, maxit=300)
    assert info["status"] == "OK"
    assert np.linalg.norm(b - A @ x.cpu().numpy()) / np.linalg.norm(b) < 1e-8
    S.set_tuning([])
    assert S.tuning() == []
    assert np.array_equal(S.apply(_cu(r), 0).cpu().numpy(), z0)


@pytest.mark.parametrize("waves", [4, 16])
@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
def test_every_shape_matches_oracle(case, variant, waves):
    # every coarse sweep at one variant (each level has five: the planned
    # shape, unsplit, and the splits over the other targets), every smoother /
    # basis product at the given waves
    p, A, b, H, S, _ = case
    levels = S.sizes()["coarse_levels"]
    recs = [{"kind": k, "index": l, "variant": variant, "waves": waves} for k in (0, 1) for l in range(levels)]
    recs += [{"kind": 2, "index": i, "variant": 0, "waves": waves} for i in range(_set_launches(S))]
    S.set_tuning(recs)
    for seed in (10, 12):
        r = synth.random_vector(A.shape[0], seed)
        z = S.apply(_cu(r), 0).cpu().numpy()
        assert _rel(z, H.apply(r)) <= 1e-12, (variant, waves, _rel(z, H.apply(r)))
        for which, op in ((1, H.apply_MG), (3, H.apply_Mzeta), (4, H.apply_Mg)):
            zw = S.apply(_cu(r), which).cpu().numpy()
            assert _rel(zw, op(r)) <= 1e-12, (variant, waves, which)
    S.set_tuning([])


def test_pinned_shapes_reproduce_bits(case):
    # a second handle given the first one's records gives the same bits
    p, A, b, H, S, (sysm, part) = case
    from paper_2509_19777_amd import hplmm as hp
    recs = S.autotune(reps=2)
    S2 = hp.Solver(sysm, part, n_mortar=4)
    S2.setup()
    S2.set_tuning(recs)
    r = _cu(synth.random_vector(A.shape[0], 5))
    assert np.array_equal(S.apply(r, 0).cpu().numpy(), S2.apply(r, 0).cpu().numpy())
    x1, i1 = S.solve(rtol=1e-8, restart=30, maxit=300)
    x2, i2 = S2.solve(rtol=1e-8, restart=30, maxit=300)
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    S.set_tuning([])


def test_graphs_follow_new_shapes(case):
    # graphs captured with the default shapes are dropped by set_tuning: the
    # solve with new shapes equals its eager counterpart, on each replay
    p, A, b, H, S, _ = case
    S.set_tuning([])
    S.use_graphs(True)
    S.solve(rtol=1e-8, restart=50, maxit=300)          # captures with the defaults
    levels = S.sizes()["coarse_levels"]
    recs = [{"kind": k, "index": l, "variant": 1, "waves": 16} for k in (0, 1) for l in range(levels)]
    S.set_tuning(recs)
    S.use_graphs(False)
    xe, ie = S.solve(rtol=1e-8, restart=50, maxit=300)
    S.use_graphs(True)
    for _ in range(3):
        xg, ig = S.solve(rtol=1e-8, restart=50, maxit=300)
        assert ig["iters"] == ie["iters"]
        assert np.array_equal(xg.cpu().numpy(), xe.cpu().numpy())
    S.set_tuning([])


def test_bad_records_restore_defaults(case):
    p, A, b, H, S, _ = case
    from paper_2509_19777_amd.hplmm import HplmmError
    r = _cu(synth.random_vector(A.shape[0], 7))
    S.set_tuning([])
    z0 = S.apply(r, 0).cpu().numpy()
    for bad in ({"kind": 0, "index": 0, "variant": 0, "waves": 8},
                {"kind": 0, "index": 999, "variant": 0, "waves": 4},
                {"kind": 1, "index": 0, "variant": 99, "waves": 4},
                {"kind": 2, "index": _set_launches(S), "variant": 0, "waves": 4},
                {"kind": 5, "index": 0, "variant": 0, "waves": 4}):
        with pytest.raises(HplmmError):
            S.set_tuning([{"kind": 2, "index": 0, "variant": 0, "waves": 16}, bad])
        assert S.tuning() == []
        assert np.array_equal(S.apply(r, 0).cpu().numpy(), z0)


def test_autotune_before_setup_is_state_error(case):
    p, A, b, H, S, (sysm, part) = case
    from paper_2509_19777_amd import hplmm as hp
    S3 = hp.Solver(sysm, part, n_mortar=4)
    with pytest.raises(hp.HplmmError) as e:
        S3.autotune()
    assert hp.STATUS[e.value.code] == "E_STATE"
