"""Pins of the oracle's reduced-precision emulation (test infrastructure for
the reduced-precision smoother parity tests).

* bfloat16 rounding: round-to-nearest-even on exact halfway cases, and the
  unit roundoff 2^-8 of an 8-bit significand as the relative error bound;
* the inverse-form emulation with no rounding (storage "f64") is exactly the
  local solve A^-1 r of every grain and contact grid, checked against
  Cholesky solves (a transposed product such as W W^T instead of W^T W, a
  wrong block or a missing contact grid fails it);
* with rounding, both forms stay within the bound their storage precision
  allows (kappa u) of the exact local solves, and the stored S is symmetric;
* the inverse form's S is the Gram matrix of the rounded inverse factor: on
  blocks with condition numbers past 1/u_bf16 it stays positive definite,
  where rounding W^T W itself entrywise to bfloat16 turns some block
  indefinite (so the emulation is not that simpler reading), and every S is
  the FP32 rounding of an exact Gram sum (its entries are FP32 values).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fem, hplmm as oh, precision as prec
from paper_2509_19777_amd import synth


def test_bf16_rounding():
    one = 1.0
    assert prec.round_bf16(np.array([one]))[0] == 1.0
    # halfway between 1 and 1 + 2^-7: ties to the even significand, 1
    assert prec.round_bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    # halfway between 1 + 2^-7 and 1 + 2^-6: ties to even, 1 + 2^-6
    assert prec.round_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6
    assert prec.round_bf16(np.array([-(1.0 + 3 * 2.0 ** -8)]))[0] == -(1.0 + 2.0 ** -6)
    x = np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).uniform(-5, 5, 10000)
    r = prec.round_bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))
    assert np.array_equal(prec.round_f32(x), x.astype(np.float32).astype(np.float64))


@pytest.fixture(scope="module")
def case():
    p = synth.config_pores(12, 4, seed=3)
    A, b, mesh = fem.assemble(p)
    H = oh.HPLMM(p, A=A, b=b, mesh=mesh, n=2)
    return A.tocsr(), H


def _exact(H, r):
    zg = np.zeros_like(r)
    for d in H.grain_dofs:
        if d.size:
            zg[d] = sla.cho_solve(sla.cho_factor(H.A[d][:, d].toarray(), lower=True), r[d])
    zc = np.zeros_like(r)
    for d in H.contact_dofs:
        zc[d] += sla.cho_solve(sla.cho_factor(H.A[d][:, d].toarray(), lower=True), r[d])
    return zg, zc


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_unrounded_inverse_form_is_the_local_solve(case):
    A, H = case
    L = prec.LowPrecisionSmoother(H, "f64", form="inverse")
    r = synth.random_vector(A.shape[0], 4)
    zg, zc = _exact(H, r)
    assert _rel(L.apply_grains(r), zg) <= 1e-12
    assert _rel(L.apply_contacts(r), zc) <= 1e-12


@pytest.mark.parametrize("form", ["factors", "inverse"])
@pytest.mark.parametrize("precision, bound", [("f32", 1e-3), ("bf16", 0.1)])
def test_rounded_forms_stay_within_their_precision(case, form, precision, bound):
    A, H = case
    L = prec.LowPrecisionSmoother(H, precision, form=form)
    r = synth.random_vector(A.shape[0], 5)
    zg, zc = _exact(H, r)
    eg, ec = _rel(L.apply_grains(r), zg), _rel(L.apply_contacts(r), zc)
    assert eg <= bound and ec <= bound, (eg, ec)
    # and the rounding is visible: not the unrounded operator
    assert eg > 1e-12 and ec > 1e-12
    if form == "inverse":
        for S in L.grain_S + L.contact_S:
            if S is not None:
                assert np.array_equal(S, S.T)


def test_inverse_form_is_gram_of_rounded_factor():
    # one synthetic SPD block with condition number 1e5 (eigenvalues spread
    # logarithmically, seeded orthogonal basis) and one from a real problem
    import scipy.sparse as sp
    from types import SimpleNamespace
    n = 60
    Q, _ = np.linalg.qr(np.random.default_rng(7).standard_normal((n, n)))
    Ab = (Q * np.logspace(0, 5, n)) @ Q.T
    Ab = 0.5 * (Ab + Ab.T)
    p = synth.config_pores(8, 4, seed=11, porosity=0.2)
    A2, b2, mesh2 = fem.assemble(p)
    d2 = np.arange(min(90, A2.shape[0]))
    A = sp.block_diag([sp.csr_matrix(Ab), A2.tocsr()[d2][:, d2]], format="csr")
    d1, d2 = np.arange(n), n + np.arange(d2.size)
    fake = SimpleNamespace(A=A, grain_dofs=[d1], grain_chol=[sla.cho_factor(Ab, lower=True)], contact_dofs=[d2])
    L = prec.LowPrecisionSmoother(fake, "bf16", form="inverse")
    for d, S, Wp in ((d1, L.grain_S[0], L.grain_Wp[0]), (d2, L.contact_S[0], L.contact_Wp[0])):
        assert np.array_equal(S, prec.round_f32(S))            # kept in FP32
        assert np.array_equal(Wp, prec.round_bf16(Wp))         # the factor is bfloat16
        assert np.linalg.eigvalsh(S).min() > 0.0               # Gram: positive definite
        # S is the FP32 rounding of the Gram sum of the bfloat16 factor
        assert np.array_equal(S, prec.round_f32(Wp.T @ Wp))
    # rounding W^T W itself entrywise would make the ill-conditioned block indefinite
    W = sla.solve_triangular(np.linalg.cholesky(Ab), np.eye(n), lower=True)
    assert np.linalg.eigvalsh(prec.round_bf16(W.T @ W)).min() < 0.0
