"""Stress recovery on the GPU (hplmm_voxel_fields) against the oracle, and
the first-pass error metric of Eq. 28 built from it.

Tolerances: sigma^t and centroid displacements 1e-12 relative to the largest
value (a few dozen FP64 operations per voxel; the Jacobi eigenvalue range
agrees with LAPACK's to ~1e-15 relative to the matrix norm); E_2 values
1e-6 relative (they compare first-pass fields whose own parity bar is 1e-12
against an FGMRES reference solved to 1e-12 on the GPU and a direct solve in
the oracle).
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


def _grid(p):
    from paper_2509_19777_amd import hplmm as hp
    sysm, part = hp.build_problem(p)
    return hp.VoxelGrid(p, sysm), sysm, part


@pytest.mark.parametrize("cfg", ["pores16", "grf64"])
def test_voxel_fields_match_oracle(cfg):
    _torch()
    from oracle import fem, stress
    p = synth.config_pores(16, 4, seed=1) if cfg == "pores16" else synth.config_grf(64, 8, seed=2, n_mortar=4)
    g, sysm, _ = _grid(p)
    mesh = fem.Mesh(p.solid)
    assert np.array_equal(mesh.xyz.astype(np.int32).ravel(), sysm.node_xyz)   # same numbering
    x = synth.random_vector(3 * sysm.n_nodes, 31)
    st, uc = g.fields(_cu(x))
    st, uc = st.cpu().numpy(), uc.cpu().numpy()
    _, st_o, uc_o, vox = stress.voxel_fields(p, mesh, x)
    assert np.abs(st[vox] - st_o).max() <= 1e-12 * np.abs(st_o).max()
    assert np.abs(uc[vox] - uc_o).max() <= 1e-12 * np.abs(uc_o).max()
    void = np.ones(st.size, dtype=bool)
    void[vox] = False
    assert np.all(st[void] == 0.0) and np.all(uc[void] == 0.0)


def test_linear_field_closed_form():
    # u = (0, 0, c z) vanishes on the clamped plane: sigma^t = E mu c on every
    # solid voxel (principal stresses lam c, lam c, (lam + 2 mu) c)
    _torch()
    p = synth.config_pores(16, 4, seed=1)
    g, sysm, _ = _grid(p)
    c = 0.003
    xyz = sysm.node_xyz.reshape(-1, 3)
    x = np.zeros(3 * sysm.n_nodes)
    x[2::3] = c * xyz[:, 2]
    st, uc = g.fields(_cu(x))
    st, uc = st.cpu().numpy(), uc.cpu().numpy()
    s = p.solid.ravel().astype(bool)
    mu = 1.0 / (2.0 * (1.0 + p.nu))
    assert np.allclose(st[s], p.E.ravel()[s] * mu * c, rtol=1e-12)
    k = np.arange(s.size) // (16 * 16)
    assert np.allclose(uc[s, 2], c * (k[s] + 0.5), rtol=1e-13)


def test_bad_arguments():
    _torch()
    from paper_2509_19777_amd import hplmm as hp
    p = synth.config_pores(16, 4, seed=1)
    g, sysm, _ = _grid(p)
    x = _cu(np.zeros(3 * sysm.n_nodes))
    for nu in (0.5, -1.0, float("nan")):
        g.nu = nu
        with pytest.raises(hp.HplmmError):
            g.fields(x)
    g.nu = p.nu
    g.dims = (0, 16, 16)
    with pytest.raises(hp.HplmmError):
        g.fields(x)


@pytest.mark.parametrize("n", [1, 4])
def test_first_pass_error_matches_oracle(n):
    # E_2 of x_aprx = M_G^-1 b against the converged solution, both ways
    _torch()
    import scipy.sparse.linalg as spla
    from oracle import fem, hplmm as oh, stress
    from paper_2509_19777_amd import hplmm as hp, variants
    p = synth.config_pores(16, 4, seed=1)
    A, b, mesh = fem.assemble(p)
    H = oh.HPLMM(p, A=A, b=b, mesh=mesh, n=n)
    xs = spla.spsolve(A.tocsc(), b)
    xa = H.apply_MG(b)
    _, st_s, u_s, _ = stress.voxel_fields(p, mesh, xs)
    _, st_a, u_a, _ = stress.voxel_fields(p, mesh, xa)
    e_sig_o, e_u_o = stress.e2_error(st_a, st_s), stress.e2_error(u_a, u_s)

    sysm, part = hp.build_problem(p)
    S = hp.Solver(sysm, part, n_mortar=n)
    S.setup()
    g = hp.VoxelGrid(p, sysm)
    xg, info = S.solve(rtol=1e-12, restart=50, maxit=1000)
    assert info["status"] == "OK"
    errs = variants.first_pass_errors(S, g, xg)
    assert abs(errs["E2_sigma_t"] - e_sig_o) <= 1e-6 * e_sig_o
    assert abs(errs["E2_u"] - e_u_o) <= 1e-6 * e_u_o


def test_variants_sweep_runs_small():
    # the sweep tool end to end on a small case: records for every (n, w_zeta),
    # the first pass improves from n = 1 (PLMM) to n = 4 under shear
    _torch()
    import dataclasses
    from paper_2509_19777_amd import variants
    p = dataclasses.replace(synth.config_grf(16, 8, seed=2, n_mortar=4), traction=variants.LOADS["shear"])
    recs = [variants.run_case(p, n, 1, reps=1) for n in (1, 4)]
    for r in recs:
        assert r["status"] == "OK" and r["exact_rel_res"] <= 1.01e-11
        assert 0.0 < r["E2_u"] < 1.0 and 0.0 < r["E2_sigma_t"] < 1.0
    assert recs[1]["E2_sigma_t"] < recs[0]["E2_sigma_t"]
