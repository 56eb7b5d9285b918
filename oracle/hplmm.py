"""Oracle: the algebraic hPLMM preconditioner, built literally.  TEST
INFRASTRUCTURE ONLY.

Follows Sec. 4 of the paper:

* Eq. (16): M^-1 = M_G^-1 + M_L^-1 (I - A M_G^-1), M_G applied first.
* Eq. (17): M_L with n_st stages of a base smoother; n_st = 1 with the
  contact-grain smoother (Sec. 5), so M_L = M_CG.
* Eq. (18)-(19): M_G^-1 = P^ (R^ A P^)^-1 R^, R^ = P^T, P^ = W Q P.
* Eq. (20): W groups fine dofs by grain grid, then by contact interface.
* Eq. (21): Q = diag(I, Q^o), Q^o built from the mortar functions.
* Eq. (22): the reduced matrix A_M = Q^T A Q with blocks A_gg, Abar_gm, ...
* Eq. (23)-(24): P = [[B, C], [I, O]], correction vectors
  c^{g_i} = (A_gi)^-1 b^{g_i}, shape vectors p_k^{g_i} = -(A_gi)^-1 Abar_{g_i m_j}
  R_m^{m_j} e_k on the grains sharing the interface of mortar node m_j.
* Eq. (25)-(26): M_CG^-1 = M_zeta^-1 + M_g^-1 (I - A M_zeta^-1), with the
  additive-Schwarz sums over grain grids and over contact grids.

Readings:
* R2: B = -A_gg^-1 Abar_gm over all grains.  A grain interior node only
  touches interface nodes whose grain set contains that grain, so
  Abar_{g_i m_j} vanishes unless g_i is in G^{c_t}; this equals Eq. (23c).
* R3: correction vectors use the right-hand side b given at set-up; a grain
  whose b^{g_i} is identically zero (or whose interior is empty) gets no
  column, since a zero column would make R^ A P^ singular (the paper notes
  c^{g_i} vanishes on unloaded grains).
* R4: the grain-grid smoother blocks are the grain interiors, the same
  A_gi as in P (the paper: both local systems use A_gi).
* The coarse matrix R^ A P^ is formed as the sparse triple product and
  factored densely (Cholesky).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem
from . import mortar as mortar_mod
from . import partition as part_mod
from . import precision as prec


def _dofs(nodes):
    nodes = np.asarray(nodes, dtype=np.int64)
    return (3 * nodes[:, None] + np.arange(3)).ravel()


class HPLMM:
    """Set-up and application of the hPLMM preconditioner for one problem.

    Attributes after construction:
      A, b, mesh, part           fine system and decomposition
      W, Q, Pr, Phat             the matrices of Eq. (19)-(23) (scipy sparse)
      B_blocks[i], c_vec[i]      per-grain shape block and correction vector
      Acoarse                    R^ A P^ (dense)
      n_mortar_dofs, corr_grains columns of P^: mortar dofs, then corrections
    """

    def __init__(self, problem, A=None, b=None, mesh=None, n=None, beta=None, w_zeta=None,
                 use_rhs=True, smoother_precision="f64", tile=64, mortar_kind="gaussian", smoother_form="factors"):
        if A is None:
            A, b_asm, mesh = fem.assemble(problem)
            if b is None:
                b = b_asm
        self.problem = problem
        self.A = A.tocsr()
        self.b = None if b is None else np.asarray(b, dtype=float)
        self.mesh = mesh
        self.n = problem.n_mortar if n is None else n
        self.beta = problem.beta if beta is None else beta
        self.w_zeta = problem.w_zeta if w_zeta is None else w_zeta
        self.N = self.A.shape[0]
        P = part_mod.classify(problem, mesh)
        part_mod.contact_grids(P, mesh, self.w_zeta)
        mortar_mod.build_mortars(P, mesh, self.n, self.beta, kind=mortar_kind, A=self.A)
        self.part = P
        self.smoother_precision = smoother_precision
        self.smoother_form = smoother_form
        self.tile = tile
        self._build_W_Q()
        self._build_P(use_rhs)
        self._build_coarse()
        self._build_smoothers()

    # ---- Eq. (20)-(21): permutation W and reduction Q --------------------
    def _build_W_Q(self):
        P = self.part
        grain_dofs = [_dofs(nodes) for nodes in P.grain_nodes]
        iface_dofs = [_dofs(nodes) for nodes in P.iface_nodes]
        self.grain_dofs, self.iface_dofs = grain_dofs, iface_dofs
        perm = np.concatenate(grain_dofs + iface_dofs) if (grain_dofs or iface_dofs) else np.zeros(0, int)
        assert perm.size == self.N and np.unique(perm).size == self.N, "every dof in exactly one block"
        self.Ngf = int(sum(d.size for d in grain_dofs))
        self.Ncf = int(sum(d.size for d in iface_dofs))
        # x^ = W x : W[orig, permuted] = 1
        self.W = sp.csr_matrix((np.ones(self.N), (perm, np.arange(self.N))), shape=(self.N, self.N))
        # Q^o = blockdiag_c M^c (Eq. 21): rows 3*v+g of the interface block,
        # columns moff_c + 3*i + gamma; M^c = H_c (x) I_3 for Gaussian mortars
        rows, cols, vals = [], [], []
        roff, coff = 0, 0
        self.moff = []
        for c, M in enumerate(P.M):
            N3, n3 = M.shape
            self.moff.append(coff)
            r, q = np.nonzero(M)
            rows.extend((roff + r).tolist())
            cols.extend((coff + q).tolist())
            vals.extend(M[r, q].tolist())
            roff += N3
            coff += n3
        self.Nmo = coff
        Qo = sp.csr_matrix((vals, (rows, cols)), shape=(self.Ncf, self.Nmo))
        self.Qo = Qo
        self.Q = sp.block_diag([sp.identity(self.Ngf, format="csr"), Qo], format="csr")

    # ---- Eq. (22)-(24): reduced system and prolongation P ---------------
    def _build_P(self, use_rhs):
        A = self.A
        Aperm = (self.W.T @ A @ self.W).tocsr()
        Ngf = self.Ngf
        self.A_gg = Aperm[:Ngf, :Ngf]
        A_gc = Aperm[:Ngf, Ngf:]
        self.Abar_gm = (A_gc @ self.Qo).tocsr()           # Eq. (22) block
        bperm = None if self.b is None else self.W.T @ self.b
        # per-grain factorisations and solves
        self.grain_chol = []
        self.B_blocks, self.c_vec, self.corr_grains = [], [], []
        b_rows, b_cols, b_vals = [], [], []
        goff = 0
        self.goff = []
        for i, dofs in enumerate(self.grain_dofs):
            ni = dofs.size
            self.goff.append(goff)
            if ni == 0:
                self.grain_chol.append(None)
                self.B_blocks.append(None)
                self.c_vec.append(None)
                continue
            Ai = self.A_gg[goff:goff + ni, goff:goff + ni].toarray()
            ch = sla.cho_factor(Ai, lower=True)
            self.grain_chol.append(ch)
            Abar_i = self.Abar_gm[goff:goff + ni].toarray()
            cols = np.flatnonzero(np.any(Abar_i != 0.0, axis=0))
            Bi = -sla.cho_solve(ch, Abar_i[:, cols])
            self.B_blocks.append((cols, Bi))
            b_rows.append(np.repeat(np.arange(goff, goff + ni), cols.size))
            b_cols.append(np.tile(cols, ni))
            b_vals.append(Bi.ravel())
            if use_rhs and bperm is not None:
                bi = bperm[goff:goff + ni]
                if np.any(bi != 0.0):
                    self.c_vec.append(sla.cho_solve(ch, bi))
                    self.corr_grains.append(i)
                else:
                    self.c_vec.append(None)
            else:
                self.c_vec.append(None)
            goff += ni
        cat = (lambda L, dt: np.concatenate(L) if L else np.zeros(0, dt))
        self.B = sp.csr_matrix((cat(b_vals, float), (cat(b_rows, int), cat(b_cols, int))),
                               shape=(Ngf, self.Nmo))
        ncorr = len(self.corr_grains)
        rows, cols, vals = [], [], []
        for j, i in enumerate(self.corr_grains):
            o = self.goff[i]
            ci = self.c_vec[i]
            rows.extend(range(o, o + ci.size))
            cols.extend([j] * ci.size)
            vals.extend(ci)
        self.C = sp.csr_matrix((vals, (rows, cols)), shape=(Ngf, ncorr))
        top = sp.hstack([self.B, self.C])
        bot = sp.hstack([sp.identity(self.Nmo), sp.csr_matrix((self.Nmo, ncorr))])
        self.Pr = sp.vstack([top, bot]).tocsr()             # Eq. (23a)
        self.Phat = (self.W @ self.Q @ self.Pr).tocsr()      # Eq. (19)
        self.ncorr = ncorr

    # ---- Eq. (18): coarse operator ---------------------------------------
    def _build_coarse(self):
        self._coarse_operator()
        self._coarse_factor()

    def _coarse_operator(self):
        Ph = self.Phat
        self.Acoarse = (Ph.T @ self.A @ Ph).toarray()

    def _coarse_factor(self):
        self.coarse_chol = sla.cho_factor(self.Acoarse, lower=True)

    # ---- Eq. (26): local blocks of the smoothers -------------------------
    def _build_smoothers(self):
        A = self.A
        self.contact_dofs = [_dofs(nodes) for nodes in self.part.contact_nodes]
        self.contact_chol = []
        for d in self.contact_dofs:
            Az = A[d][:, d].toarray()
            self.contact_chol.append(sla.cho_factor(Az, lower=True))
        self.lowp = None
        if self.smoother_precision != "f64":
            self.lowp = prec.LowPrecisionSmoother(self, self.smoother_precision, self.tile, self.smoother_form)

    # ---- applications -----------------------------------------------------
    def apply_MG(self, r):
        """M_G^-1 r = P^ (R^ A P^)^-1 P^T r   (Eq. 18)."""
        rc = self.Phat.T @ r
        return self.Phat @ sla.cho_solve(self.coarse_chol, rc)

    def coarse_solution(self, r):
        return sla.cho_solve(self.coarse_chol, self.Phat.T @ r)

    def apply_Mg(self, r):
        """Grain-grid additive Schwarz, Eq. (26) left (disjoint blocks)."""
        if self.lowp is not None:
            return self.lowp.apply_grains(r)
        z = np.zeros_like(r)
        for dofs, ch in zip(self.grain_dofs, self.grain_chol):
            if ch is None:
                continue
            z[dofs] = sla.cho_solve(ch, r[dofs])
        return z

    def apply_Mzeta(self, r):
        """Contact-grid additive Schwarz, Eq. (26) right (overlapping blocks,
        summed in contact-grid order)."""
        if self.lowp is not None:
            return self.lowp.apply_contacts(r)
        z = np.zeros_like(r)
        for dofs, ch in zip(self.contact_dofs, self.contact_chol):
            z[dofs] += sla.cho_solve(ch, r[dofs])
        return z

    def apply_MCG(self, r):
        """Contact-grain smoother, Eq. (25)."""
        z2 = self.apply_Mzeta(r)
        return z2 + self.apply_Mg(r - self.A @ z2)

    def apply_ML(self, r, n_st=1):
        """Eq. (17) with base smoother M_CG and n_st stages."""
        z = np.zeros_like(r)
        res = r.copy()
        for _ in range(n_st):
            dz = self.apply_MCG(res)
            z += dz
            res = res - self.A @ dz
        return z

    def apply(self, r):
        """M^-1 r, Eq. (16): coarse first, then the smoother."""
        z1 = self.apply_MG(r)
        return z1 + self.apply_ML(r - self.A @ z1)

    def first_pass(self):
        """x_aprx = M_G^-1 b (Sec. 6.1)."""
        return self.apply_MG(self.b)

    # ---- diagnostics -------------------------------------------------------
    def max_local_condition(self):
        """Largest 2-norm condition number among grain and contact blocks."""
        k = 0.0
        for ch in self.grain_chol + self.contact_chol:
            if ch is None:
                continue
            L = np.tril(ch[0])
            s = np.linalg.svd(L, compute_uv=False)
            k = max(k, (s[0] / s[-1]) ** 2)
        return k


class LocalSmoothers:
    """The two additive-Schwarz sums of Eq. (26) and their composition
    Eq. (25), without the coarse space: grain interiors (R4) and contact grids
    (R5) classified and factored exactly as in HPLMM, so that the smoother of
    a problem too large for the dense coarse factor can still be checked
    block by block.  FP64 only."""

    def __init__(self, problem, A, mesh, w_zeta=None):
        self.A = A.tocsr()
        w = problem.w_zeta if w_zeta is None else w_zeta
        P = part_mod.classify(problem, mesh)
        part_mod.contact_grids(P, mesh, w)
        self.part = P
        self.grain_dofs = [_dofs(nodes) for nodes in P.grain_nodes]
        self.contact_dofs = [_dofs(nodes) for nodes in P.contact_nodes]
        self.grain_chol = [sla.cho_factor(self.A[d][:, d].toarray(), lower=True) if d.size else None
                           for d in self.grain_dofs]
        self.contact_chol = [sla.cho_factor(self.A[d][:, d].toarray(), lower=True) for d in self.contact_dofs]

    def apply_Mg(self, r):
        z = np.zeros_like(r)
        for dofs, ch in zip(self.grain_dofs, self.grain_chol):
            if ch is not None:
                z[dofs] = sla.cho_solve(ch, r[dofs])
        return z

    def apply_Mzeta(self, r):
        z = np.zeros_like(r)
        for dofs, ch in zip(self.contact_dofs, self.contact_chol):
            z[dofs] += sla.cho_solve(ch, r[dofs])
        return z

    def apply_MCG(self, r):
        z2 = self.apply_Mzeta(r)
        return z2 + self.apply_Mg(r - self.A @ z2)

