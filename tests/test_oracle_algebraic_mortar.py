"""Pins of the oracle's algebraic mortars (Eq. 9 in the algebraic form of
the Remark after Eq. 22) against independent characterisations:

* each column is the minimiser of the interface energy eta^T A_cc eta under
  the mortar-node constraints, computed here through the KKT system with
  Lagrange multipliers (a different linear system from the elimination the
  oracle performs);
* perturbing the free dofs never lowers that energy;
* the constrained rows are exactly the identity, and with every interface
  node a mortar node the block is the identity;
* the coarse preconditioner built with these mortars is still an
  A-orthogonal projector (Eq. 18 does not depend on the mortar kind).
"""
import numpy as np
import pytest

from oracle import fem, hplmm as oh, mortar, partition
from paper_2509_19777_amd import synth


@pytest.fixture(scope="module")
def case():
    p = synth.config_pores(16, 4, seed=1)
    A, b, mesh = fem.assemble(p)
    P = partition.classify(p, mesh)
    return p, A.tocsr(), b, mesh, P


def _iface(case, c, n):
    p, A, b, mesh, P = case
    nodes = P.iface_nodes[c]
    d = (3 * np.asarray(nodes, dtype=np.int64)[:, None] + np.arange(3)).ravel()
    Acc = A[d][:, d].toarray()
    idx = mortar.place_mortars(mesh.xyz[nodes], min(n, len(nodes)))
    return Acc, idx


def _big_ifaces(case, k=4):
    P = case[4]
    sizes = np.array([len(x) for x in P.iface_nodes])
    return list(np.argsort(-sizes)[:k])


@pytest.mark.parametrize("n", [1, 2, 4])
def test_columns_solve_the_kkt_system(case, n):
    for c in _big_ifaces(case):
        Acc, idx = _iface(case, c, n)
        M = mortar.algebraic_block(Acc, idx)
        N3, nK = Acc.shape[0], 3 * len(idx)
        C = np.zeros((nK, N3))
        for i, m in enumerate(idx):
            for g in range(3):
                C[3 * i + g, 3 * m + g] = 1.0
        KKT = np.block([[Acc, C.T], [C, np.zeros((nK, nK))]])
        rhs = np.vstack([np.zeros((N3, nK)), np.eye(nK)])
        sol = np.linalg.solve(KKT, rhs)[:N3]
        assert np.abs(M - sol).max() <= 1e-10 * max(1.0, np.abs(sol).max())


def test_energy_is_minimal_and_constraints_exact(case):
    rng = np.random.default_rng(0)
    for c in _big_ifaces(case):
        Acc, idx = _iface(case, c, 4)
        M = mortar.algebraic_block(Acc, idx)
        K = np.array([3 * m + g for m in idx for g in range(3)])
        assert np.array_equal(M[K], np.eye(K.size))
        F = np.setdiff1d(np.arange(Acc.shape[0]), K)
        for j in range(M.shape[1]):
            e0 = M[:, j] @ Acc @ M[:, j]
            for _ in range(5):
                d = np.zeros(Acc.shape[0])
                d[F] = 1e-3 * rng.standard_normal(F.size)
                assert (M[:, j] + d) @ Acc @ (M[:, j] + d) >= e0 - 1e-12 * abs(e0)


def test_all_nodes_mortar_gives_identity(case):
    c = _big_ifaces(case, 1)[0]
    Acc, _ = _iface(case, c, 10 ** 6)
    N = Acc.shape[0] // 3
    M = mortar.algebraic_block(Acc, list(range(N)))
    assert np.array_equal(M, np.eye(3 * N))


def test_coarse_preconditioner_is_a_projector(case):
    p, A, b, mesh, P = case
    H = oh.HPLMM(p, A=A, b=b, mesh=mesh, n=2, mortar_kind="algebraic")
    v = synth.random_vector(A.shape[0], 3)
    Pv = H.apply_MG(A @ v)
    PPv = H.apply_MG(A @ Pv)
    assert np.linalg.norm(PPv - Pv) <= 1e-10 * np.linalg.norm(Pv)
    # the algebraic Q^o differs from the Gaussian one but spans the interface
    # values at the mortar nodes in the same way
    G = oh.HPLMM(p, A=A, b=b, mesh=mesh, n=2)
    assert H.Qo.shape == G.Qo.shape
    assert np.abs((H.Qo - G.Qo).toarray()).max() > 1e-3
