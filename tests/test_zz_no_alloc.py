"""hplmm_apply_noalloc (static split-row scratch, no allocation) against
hplmm_apply, through the C ABI: the same kernels at the same launch shapes,
so the results must agree bit for bit.  Two problems in a row, the second
smaller, so the second call finds the first call's partial sums in the
shared buffer."""
import numpy as np
import pytest

from paper_2509_19777_amd import synth

pytestmark = pytest.mark.gpu


def _solver(n_vox, seed):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_19777_amd import hplmm as hp
    p = synth.config_pores(n_vox, 4, seed=seed)
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=2)
    S.setup()
    return S


def _check(S, seed):
    import torch
    n = 3 * S.sizes()["n_nodes"]
    part = S.split_scratch()
    assert part > 0, "the coarse sweeps of this case must use split rows"
    r = torch.from_numpy(synth.random_vector(n, seed)).cuda()
    for which in range(5):
        ref = S.apply(r, which=which)
        out = torch.full_like(r, float("nan"))
        S.apply_noalloc(r, which=which, out=out)
        torch.cuda.synchronize()
        print(f"no-alloc apply n={n} which={which}", flush=True)
        assert torch.equal(out, ref), f"which={which}: max diff {(out - ref).abs().max().item():.3e}"


def test_noalloc_apply_matches_apply_on_two_problems():
    big = _solver(16, 1)
    small = _solver(12, 3)
    assert 3 * small.sizes()["n_nodes"] < 3 * big.sizes()["n_nodes"]
    _check(big, 20)
    _check(small, 21)
    # and back: the smaller call's leftovers in the shared buffer do not matter
    _check(big, 22)


def test_noalloc_apply_rejects_bad_arguments():
    import torch
    from paper_2509_19777_amd import hplmm as hp
    S = _solver(12, 3)
    n = 3 * S.sizes()["n_nodes"]
    r = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(hp.HplmmError):
        S.apply_noalloc(r, which=5, out=torch.empty_like(r))
    with pytest.raises(hp.HplmmError):
        S.apply_noalloc(r, which=0, out=r)
