"""Oracle: emulation of the reduced-precision smoother.  TEST INFRASTRUCTURE
ONLY.

The paper runs everything in (presumably) FP64.  The reduced-precision
variant keeps the coarse space in FP64 and stores the smoother operators at
lower precision.  This module rounds values at the same storage points, with
round-to-nearest-even, and performs the arithmetic in between in FP64 (grain
blocks) or FP32 (contact blocks), as the variant prescribes:

* grain blocks: the FP64 Cholesky factor L_i of A_gi is inverted in FP64,
  W_i = L_i^-1, and W_i is rounded to the storage precision; the smoother is
  z = W_i^T (W_i r) evaluated in FP64 on the rounded W_i;
* contact blocks: A_zeta is rounded to FP32, factored and inverted in FP32,
  and the FP32 inverse factor is rounded to the storage precision.

That is the factor form (form="factors").  In the inverse form
(form="inverse") every block, grain and contact grid alike, is factored and
inverted in FP64, W is rounded to the storage precision (Wp), and the
smoother's operator is the Gram matrix S = Wp^T Wp, formed exactly (the
products of rounded values are exact in FP64, the sums carry FP64 rounding
only) and rounded once to FP32, the precision it is kept in; the smoother is
z = S r evaluated in FP64.  S is positive definite whatever the rounding of W
(the Gram matrix of a nonsingular matrix), unlike W^T W rounded entrywise.
With storage "f64" nothing is rounded: S = W^T W.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def round_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    """Round FP64 values to bfloat16 (via FP32), round-to-nearest-even."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    u = ((u + bias) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def round_to(x, precision):
    if precision == "f64":
        return np.asarray(x, dtype=np.float64)
    if precision == "f32":
        return round_f32(x)
    if precision == "bf16":
        return round_bf16(x)
    raise ValueError(precision)


class LowPrecisionSmoother:
    def __init__(self, H, precision, tile=64, form="factors"):
        self.H = H
        self.precision = precision
        self.form = form
        if form == "inverse":
            self._build_inverse()
            return
        if form != "factors":
            raise ValueError(form)
        self.grain_W = []
        for ch in H.grain_chol:
            if ch is None:
                self.grain_W.append(None)
                continue
            L = np.tril(ch[0])
            Wi = sla.solve_triangular(L, np.eye(L.shape[0]), lower=True)
            self.grain_W.append(round_to(Wi, precision))
        self.contact_W = []
        for d in H.contact_dofs:
            Az = H.A[d][:, d].toarray().astype(np.float32)
            L32 = np.linalg.cholesky(Az).astype(np.float32)
            W32 = sla.solve_triangular(L32, np.eye(L32.shape[0], dtype=np.float32), lower=True)
            self.contact_W.append(round_to(W32.astype(np.float64), precision))

    def _build_inverse(self):
        def gram_of_rounded(A):
            L = np.linalg.cholesky(A)
            W = sla.solve_triangular(L, np.eye(L.shape[0]), lower=True)
            if self.precision == "f64":
                return W, W.T @ W
            Wp = round_to(W, self.precision)
            return Wp, round_f32(Wp.T @ Wp)
        g = [None if ch is None else gram_of_rounded(self.H.A[d][:, d].toarray())
             for d, ch in zip(self.H.grain_dofs, self.H.grain_chol)]
        c = [gram_of_rounded(self.H.A[d][:, d].toarray()) for d in self.H.contact_dofs]
        self.grain_Wp = [None if x is None else x[0] for x in g]
        self.grain_S = [None if x is None else x[1] for x in g]
        self.contact_Wp = [x[0] for x in c]
        self.contact_S = [x[1] for x in c]

    def apply_grains(self, r):
        z = np.zeros_like(r)
        if self.form == "inverse":
            for dofs, Si in zip(self.H.grain_dofs, self.grain_S):
                if Si is not None:
                    z[dofs] = Si @ r[dofs]
            return z
        for dofs, Wi in zip(self.H.grain_dofs, self.grain_W):
            if Wi is None:
                continue
            z[dofs] = Wi.T @ (Wi @ r[dofs])
        return z

    def apply_contacts(self, r):
        z = np.zeros_like(r)
        if self.form == "inverse":
            for dofs, Sz in zip(self.H.contact_dofs, self.contact_S):
                z[dofs] += Sz @ r[dofs]
            return z
        for dofs, Wz in zip(self.H.contact_dofs, self.contact_W):
            z[dofs] += Wz.T @ (Wz @ r[dofs])
        return z
