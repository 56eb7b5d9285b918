"""GPU parity on an irregular (Voronoi) partition of a fractured, two-phase
pore domain: subdomains of uneven size share every launch.  Same bars as the
box-partition parity tests (FP64 apply 1e-12, FGMRES within one iteration of
the oracle and 1e-8 at the oracle's iteration count)."""
import numpy as np
import pytest

from paper_2509_19777_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def uneven():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import fem, hplmm as oh
    from paper_2509_19777_amd import hplmm as hp
    p = synth.config_uneven(16, seed=5, dofs_per_cell=300, n_mortar=2)
    A, b, mesh = fem.assemble(p)
    H = oh.HPLMM(p, A=A, b=b, mesh=mesh, n=2)
    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=2)
    S.setup()
    return p, A, b, H, S


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_sizes_are_uneven(uneven):
    p, A, b, H, S = uneven
    n = [len(g) for g in H.part.grain_nodes if len(g)]
    assert max(n) >= 3 * min(n)


@pytest.mark.parametrize("which", [0, 1, 2, 3, 4])
def test_apply_parity_uneven(uneven, which):
    import torch
    p, A, b, H, S = uneven
    ops = {0: H.apply, 1: H.apply_MG, 2: H.apply_MCG, 3: H.apply_Mzeta, 4: H.apply_Mg}
    for r in (b, synth.random_vector(A.shape[0], 31)):
        z = S.apply(torch.from_numpy(r).cuda(), which).cpu().numpy()
        assert _rel(z, ops[which](r)) <= 1e-12


def test_solve_parity_uneven(uneven):
    from oracle import gmres
    p, A, b, H, S = uneven
    ro = gmres.gmres(A, b, H.apply, tol=1e-8, restart=50, flexible=True)
    x, info = S.solve(rtol=1e-8, restart=50, maxit=300)
    assert info["status"] == "OK" and abs(info["iters"] - ro.iters) <= 1
    xf, _ = S.solve(rtol=1e-8, restart=50, maxit=300, fixed_iters=ro.iters)
    assert _rel(xf.cpu().numpy(), ro.x) <= 1e-8
