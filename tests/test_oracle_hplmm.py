"""Pins of the oracle's hPLMM preconditioner (paper Sec. 4, Eqs. 16-26)
against identities the method implies, the paper's own limits (n = 1 is
PLMM; n = number of interface nodes makes the first pass exact, App. B), the
error-propagation split of Eq. 29, and literal dense brute force."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import fem, hplmm
from paper_2509_19777_amd import synth


@pytest.fixture(scope="module")
def small():
    p = synth.config_pores(12, 4, seed=7)
    A, b, mesh = fem.assemble(p)
    H = hplmm.HPLMM(p, A=A, b=b, mesh=mesh, n=2)
    return p, A, b, mesh, H


@pytest.fixture(scope="module")
def tiny():
    p = synth.config_pores(8, 4, seed=11, porosity=0.2)
    A, b, mesh = fem.assemble(p)
    H = hplmm.HPLMM(p, A=A, b=b, mesh=mesh, n=2)
    return p, A, b, mesh, H


def test_harmonic_extension_identity(small):
    """A_gg B + Abar_gm = 0 (Eq. 23c: each shape vector solves its local problem)."""
    *_, H = small
    R = H.A_gg @ H.B + H.Abar_gm
    assert abs(R).max() <= 1e-12 * abs(H.Abar_gm).max()


def test_shape_vectors_literal_eq23(tiny):
    """Each column k of B built literally from Eq. (23c) with the contraction
    R_m^{m_j} e_k (Eq. 24), grain by grain, only on the grains sharing the
    interface hosting mortar node m_j."""
    p, A, b, mesh, H = tiny
    Nmo = H.Nmo
    Abar = H.Abar_gm.toarray()
    Bfull = H.B.toarray()
    # interface of every mortar dof
    iface_of_col = np.empty(Nmo, dtype=int)
    for c, H_c in enumerate(H.part.H):
        iface_of_col[H.moff[c]:H.moff[c] + 3 * H_c.shape[1]] = c
    for k in range(Nmo):
        mj = k // 3
        e = np.zeros(Nmo)
        e[k] = 1.0
        Rm = np.zeros((3, Nmo))
        Rm[:, 3 * mj:3 * mj + 3] = np.eye(3)
        ct = iface_of_col[k]
        for gi, dofs in enumerate(H.grain_dofs):
            if dofs.size == 0:
                continue
            o = H.goff[gi]
            rows = slice(o, o + dofs.size)
            if gi in H.part.iface_grains[ct]:
                Abar_gi_mj = Abar[rows, 3 * mj:3 * mj + 3]
                pk = -sla.cho_solve(H.grain_chol[gi], Abar_gi_mj @ (Rm @ e))
            else:
                pk = np.zeros(dofs.size)
            assert np.allclose(Bfull[rows, k], pk, rtol=0, atol=1e-13)


def test_coarse_operator_structure(small):
    """R^ A P^ is symmetric positive definite and its mortar x correction
    block vanishes (a consequence of the identity A_gg B + Abar_gm = 0)."""
    *_, H = small
    Ac = H.Acoarse
    assert np.allclose(Ac, Ac.T, rtol=0, atol=1e-14 * abs(Ac).max())
    assert np.linalg.eigvalsh(Ac).min() > 0
    cross = Ac[:H.Nmo, H.Nmo:]
    assert abs(cross).max() <= 1e-12 * abs(Ac).max()


def test_first_pass_is_galerkin_on_range_WQ(small):
    """M_G^-1 b equals the Galerkin solution of A x = b on range(W Q)."""
    p, A, b, mesh, H = small
    WQ = (H.W @ H.Q).tocsc()
    AM = (WQ.T @ A @ WQ).toarray()
    xq = WQ @ np.linalg.solve(AM, WQ.T @ b)
    fp = H.first_pass()
    assert np.linalg.norm(fp - xq) <= 1e-12 * np.linalg.norm(xq)


def test_coarse_preconditioner_is_A_projector(small):
    p, A, b, mesh, H = small
    v = np.random.default_rng(1).standard_normal(A.shape[0])
    y1 = H.apply_MG(A @ v)
    y2 = H.apply_MG(A @ y1)
    assert np.linalg.norm(y2 - y1) <= 1e-11 * np.linalg.norm(y1)


def test_all_nodes_as_mortars_gives_exact_first_pass(small):
    """App. B: with as many mortar nodes as interface nodes the first pass is
    the exact solution."""
    p, A, b, mesh, _ = small
    H = hplmm.HPLMM(p, A=A, b=b, mesh=mesh, n=10 ** 6)
    xs = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(H.first_pass() - xs) <= 1e-12 * np.linalg.norm(xs)


def test_plmm_limit_rigid_interfaces(small):
    """n = 1 (PLMM): every interface dof block of P^ restricted to one mortar
    is a uniform translation of that interface."""
    p, A, b, mesh, _ = small
    H = hplmm.HPLMM(p, A=A, b=b, mesh=mesh, n=1)
    assert H.Nmo == 3 * len(H.part.iface_nodes)
    Qo = H.Qo.toarray()
    assert np.array_equal(Qo, np.abs(Qo))
    assert np.array_equal(Qo.sum(axis=1), np.ones(Qo.shape[0]))
    for c, dofs in enumerate(H.iface_dofs):
        blk = Qo[:, 3 * c:3 * c + 3]
        assert np.array_equal(np.flatnonzero(blk.any(axis=1)),
                              np.arange(sum(d.size for d in H.iface_dofs[:c]),
                                        sum(d.size for d in H.iface_dofs[:c + 1])))


def test_prolongation_reproduces_translation(small):
    """Prolonging a uniform translation t on every mortar dof (correction
    coefficients 0) reproduces t on every interior node of a grain none of
    whose nodes touches the clamped plane; partition of unity of the mortars
    plus A t = 0 away from the constraint."""
    p, A, b, mesh, H = small
    t = np.array([0.3, -1.1, 0.7])
    u = np.zeros(H.Nmo + H.ncorr)
    u[:H.Nmo] = np.tile(t, H.Nmo // 3)
    x = H.Phat @ u
    for gi, nodes in enumerate(H.part.grain_nodes):
        if nodes.size == 0:
            continue
        # the grain's local problem sees the clamp if any neighbour is clamped:
        # skip grains in the bottom layer of boxes
        if mesh.xyz[nodes][:, 2].min() <= 4:
            continue
        d = (3 * nodes[:, None] + np.arange(3)).ravel()
        assert np.allclose(x[d], np.tile(t, nodes.size), rtol=0, atol=1e-12)
    for c, nodes in enumerate(H.part.iface_nodes):
        d = (3 * nodes[:, None] + np.arange(3)).ravel()
        assert np.allclose(x[d], np.tile(t, nodes.size), rtol=0, atol=1e-14)


def test_grain_smoother_local_exactness(small):
    """R_g (r - A M_g^-1 r) = 0 on every grain interior (disjoint blocks)."""
    p, A, b, mesh, H = small
    r = np.random.default_rng(2).standard_normal(A.shape[0])
    res = r - A @ H.apply_Mg(r)
    for dofs in H.grain_dofs:
        if dofs.size:
            assert np.abs(res[dofs]).max() <= 1e-12 * np.abs(r).max()


def test_smoothers_match_literal_eq26(tiny):
    """Eq. (26) with explicit 0/1 restriction matrices R_f and E_f = R_f^T."""
    p, A, b, mesh, H = tiny
    Ad = A.toarray()
    N = Ad.shape[0]
    r = np.random.default_rng(3).standard_normal(N)

    def schwarz(blocks):
        Minv = np.zeros((N, N))
        for d in blocks:
            if d.size == 0:
                continue
            R = np.zeros((d.size, N))
            R[np.arange(d.size), d] = 1.0
            Minv += R.T @ np.linalg.inv(R @ Ad @ R.T) @ R
        return Minv

    Mg = schwarz(H.grain_dofs)
    Mz = schwarz(H.contact_dofs)
    assert np.allclose(H.apply_Mg(r), Mg @ r, rtol=0, atol=1e-10 * np.abs(Mg @ r).max())
    assert np.allclose(H.apply_Mzeta(r), Mz @ r, rtol=0, atol=1e-10 * np.abs(Mz @ r).max())
    MCG = Mz + Mg @ (np.eye(N) - Ad @ Mz)               # Eq. (25)
    assert np.allclose(H.apply_MCG(r), MCG @ r, rtol=0, atol=1e-10 * np.abs(MCG @ r).max())


def test_error_propagation_split_eq29(tiny):
    """I - M^-1 A = (I - M_L^-1 A)(I - M_G^-1 A): M_G is applied first."""
    p, A, b, mesh, H = tiny
    v = np.random.default_rng(4).standard_normal(A.shape[0])
    lhs = v - H.apply(A @ v)
    w = v - H.apply_MG(A @ v)
    rhs = w - H.apply_ML(A @ w)
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(v)
    # the opposite order is a different operator (the test can tell them apart)
    w2 = v - H.apply_ML(A @ v)
    other = w2 - H.apply_MG(A @ w2)
    assert np.linalg.norm(lhs - other) > 1e-6 * np.linalg.norm(v)


def test_coarse_literal_triple_product(tiny):
    """R^ A P^ formed densely from W, Q, P equals the oracle's coarse matrix,
    and W is a permutation (W W^T = I)."""
    p, A, b, mesh, H = tiny
    W = H.W.toarray()
    assert np.array_equal(W @ W.T, np.eye(W.shape[0]))
    Ph = W @ H.Q.toarray() @ H.Pr.toarray()
    Ac = Ph.T @ A.toarray() @ Ph
    assert np.allclose(Ac, H.Acoarse, rtol=0, atol=1e-13 * abs(Ac).max())


def test_local_smoothers_without_coarse_space(tiny, small):
    """LocalSmoothers (the smoother alone, for full-size checks) against the
    literal Eq. (26) sums with explicit 0/1 restrictions on the tiny case, and
    against the full preconditioner's smoother on the small one."""
    p, A, b, mesh, H = tiny
    L = hplmm.LocalSmoothers(p, A, mesh)
    Ad = A.toarray()
    N = Ad.shape[0]
    r = np.random.default_rng(5).standard_normal(N)
    for blocks, op in ((L.grain_dofs, L.apply_Mg), (L.contact_dofs, L.apply_Mzeta)):
        M = np.zeros((N, N))
        for d in blocks:
            if d.size:
                R = np.zeros((d.size, N))
                R[np.arange(d.size), d] = 1.0
                M += R.T @ np.linalg.inv(R @ Ad @ R.T) @ R
        assert np.allclose(op(r), M @ r, rtol=0, atol=1e-10 * np.abs(M @ r).max())
    p, A, b, mesh, H = small
    L = hplmm.LocalSmoothers(p, A, mesh)
    r = np.random.default_rng(6).standard_normal(A.shape[0])
    for a, c in ((L.apply_Mg, H.apply_Mg), (L.apply_Mzeta, H.apply_Mzeta), (L.apply_MCG, H.apply_MCG)):
        assert np.array_equal(a(r), c(r))
