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


def test_bf16_inference_keeps_the_method(fresh):
    # the same network with bfloat16 operands: its shape vectors stay as
    # accurate (the error is the network's, not bfloat16's), the 1e-3 fallback
    # still keeps the exact method's iterations, and the inference time is
    # printed beside the FP32 one
    from paper_2509_19777_amd import hplmm as hp, surrogate as sgm
    p, net = fresh
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=4)
    S.setup()
    x, y, meta = hp.surrogate_samples(S)
    e32 = sgm.per_sample_error(net, x, y, 128)
    rows32 = sgm.compare(net, p, [1e-3], reps=2)
    net.set_inference_precision(16)
    try:
        e16 = sgm.per_sample_error(net, x, y, 128)
        rows16 = sgm.compare(net, p, [1e-3], reps=2)
    finally:
        net.set_inference_precision(32)
    print(json.dumps({"median_rel_err_fp32": float(np.median(e32)), "median_rel_err_bf16": float(np.median(e16)),
                      "t_infer_ms_fp32": rows32[1]["t_infer_ms"], "t_infer_ms_bf16": rows16[1]["t_infer_ms"],
                      "setup_ms_exact": rows16[0]["setup_ms"], "setup_ms_surrogate_bf16": rows16[1]["setup_ms"]}))
    assert abs(np.median(e16) - np.median(e32)) <= 0.05 * np.median(e32)
    assert rows16[1]["status"] == "OK" and rows16[1]["iters"] == rows16[0]["iters"]
