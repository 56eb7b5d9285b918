"""What the trained basis surrogate gains over the method without it, on a
fresh domain (seed 7, not among the training seeds 1000-1039), 32^3 voxels of
pores with a lognormal modulus, 8^3-voxel grains, n = 4.

Checked: the network has learned (its relative error on the fresh domain's
shape vectors is well below the 1.0 of predicting zero); with the local
residual threshold 1e-3 of the method's fallback every rejected grain gets the
exact basis, so FGMRES needs exactly the iterations of the exact set-up; with
every prediction accepted FGMRES needs more iterations.  The measured numbers
are printed (pytest -s) and recorded in the design notes."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fresh():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_19777_amd import hplmm as hp, surrogate as sgm, synth
    p = synth.config_pores_lognormal(32, 8, seed=sgm.EVAL_SEED, n_mortar=4)
    net = hp.SurrogateNet(sgm.CHANNELS, max_batch=128)
    net.set_params(np.load(sgm.DEFAULT_WEIGHTS)["params"])
    return p, net


def test_network_learned_the_shape_vectors(fresh):
    from paper_2509_19777_amd import hplmm as hp, surrogate as sgm
    p, net = fresh
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=4)
    S.setup()
    x, y, meta = hp.surrogate_samples(S)
    e = sgm.per_sample_error(net, x, y, 128)
    print(json.dumps({"samples": int(e.size), "median_rel_err": float(np.median(e)),
                      "p90_rel_err": float(np.quantile(e, 0.9))}))
    assert np.median(e) < 0.5


def test_fallback_keeps_the_method_and_acceptance_costs_iterations(fresh):
    from paper_2509_19777_amd import surrogate as sgm
    p, net = fresh
    rows = sgm.compare(net, p, [1e-3, 1e300], reps=1)
    for r in rows:
        print(json.dumps(r))
    exact, strict, loose = rows
    assert exact["status"] == "OK" and strict["status"] == "OK"
    assert strict["iters"] == exact["iters"]
    assert strict["accepted"] == 0 or strict["max_residual_accepted"] <= 1e-3
    assert loose["accepted"] > 0
    assert loose["iters"] > exact["iters"]
