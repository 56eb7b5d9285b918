"""Oracle: mortar nodes and Gaussian mortar functions.  TEST INFRASTRUCTURE
ONLY.

Follows Sec. 3.3 of the paper: mortar nodes are placed on an interface as
like-charged particles (start from the two farthest interface nodes, add nodes
one at a time by minimising the summed inverse distance to the nodes already
placed, Eq. 7, then sweep over the nodes moving each to the minimiser of its
potential with the others fixed until nothing moves), and each mortar node
carries a Gaussian mortar function normalised to a partition of unity (Eq. 8),
with beta = 4.

Readings:
* R6: nu_c = min(n, N_c).  nu_c = 1 gives the all-ones weight (PLMM); when
  nu_c = N_c the weight block is the identity (the span of the Gaussian
  weights is then the whole interface space, as the paper's appendix uses).
* R7: positions are integer lattice points; the farthest pair is the pair of
  largest squared distance with ties to the lexicographically smallest index
  pair; each greedy step takes the argmin of the potential summed over placed
  nodes in placement order, ties (relative 1e-12) to the smallest node index.
  The paper sweeps in random order; here sweeps go in mortar order, and a node
  moves only when its potential drops by more than a relative 1e-12, which
  strictly lowers the total potential, so the sweeps end (capped at 100).
* R8: the denominator of Eq. 8 uses the smallest distance from mortar node i
  to any *other* mortar node; weights act identically on the x, y, z
  components (global frame), so the Gaussian span does not depend on the
  local normal/tangent frame.
"""
from __future__ import annotations

import numpy as np

REL_TIE = 1e-12


def _potential(pos, y, others):
    s = 0.0
    for j in others:
        d2 = float(np.sum((pos[y] - pos[j]) ** 2))
        s += 1.0 / np.sqrt(d2)
    return s


def _argmin_potential(pos, candidates, placed):
    """argmin over candidates of sum_{j in placed, in order} 1/|y - x_j|;
    ties within REL_TIE of the minimum go to the smallest node index."""
    vals = []
    for y in candidates:
        if y in placed:
            continue
        vals.append((_potential(pos, y, placed), y))
    best = min(v for v, _ in vals)
    return min(y for v, y in vals if v <= best * (1.0 + REL_TIE))


def place_mortars(pos, nu, max_sweeps=100):
    """Indices (into pos) of the nu mortar nodes of one interface.

    pos: (N_c, 3) integer coordinates of the interface nodes, in the
    interface's node order.  Returns a list of length nu.
    """
    pos = np.asarray(pos, dtype=np.int64)
    N = pos.shape[0]
    if nu >= N:
        return list(range(N))
    if nu == 1:
        return [0]
    best, pair = -1, None
    for a in range(N):
        d2 = np.sum((pos[a + 1:] - pos[a]) ** 2, axis=1)
        if d2.size == 0:
            continue
        m = int(d2.max())
        if m > best:
            best = m
            pair = (a, a + 1 + int(np.flatnonzero(d2 == m)[0]))
    placed = [pair[0], pair[1]]
    while len(placed) < nu:
        placed.append(_argmin_potential(pos, range(N), placed))
    for _ in range(max_sweeps):
        moved = False
        for m in range(nu):
            others = placed[:m] + placed[m + 1:]
            cur = _potential(pos, placed[m], others)
            y = _argmin_potential(pos, range(N), others)
            if y != placed[m] and _potential(pos, y, others) < cur * (1.0 - REL_TIE):
                placed[m] = y
                moved = True
        if not moved:
            break
    return placed


def gaussian_weights(pos, mortar_idx, beta=4.0):
    """H (N_c x nu): H[v, i] = alpha_i(x_v) / sum_j alpha_j(x_v) with
    alpha_i(x) = exp(-|x - x_i|^2 / (beta * min_{j != i} |x_i - x_j|^2)) (Eq. 8)."""
    pos = np.asarray(pos, dtype=float)
    nu = len(mortar_idx)
    N = pos.shape[0]
    if nu == 1:
        return np.ones((N, 1))
    if nu >= N:
        return np.eye(N)
    xm = pos[mortar_idx]
    dmin2 = np.empty(nu)
    for i in range(nu):
        d2 = np.sum((xm - xm[i]) ** 2, axis=1)
        d2[i] = np.inf
        dmin2[i] = d2.min()
    alpha = np.empty((N, nu))
    for i in range(nu):
        alpha[:, i] = np.exp(-np.sum((pos - xm[i]) ** 2, axis=1) / (beta * dmin2[i]))
    return alpha / alpha.sum(axis=1, keepdims=True)


def algebraic_block(Acc, mortar_idx):
    """Algebraic mortar block M^{c} (3 N_c x 3 nu) of one interface, built as
    the Remark after Eq. 22 describes: column (i, gamma) holds 1 at dof gamma
    of mortar node i, 0 at every other mortar-node dof, and on the remaining
    (free) interface dofs F the values -(A_FF)^-1 A_F,(i,gamma), i.e. the
    interface-restricted operator's response to that unit constraint.

    Acc: the interface-interface block of A (3 N_c x 3 N_c, dofs 3 v + g in
    the interface's node order).  Rows of the result are 3 v + g, columns
    3 i + gamma (mortar order)."""
    Acc = np.asarray(Acc.todense() if hasattr(Acc, "todense") else Acc, dtype=float)
    N3 = Acc.shape[0]
    nu = len(mortar_idx)
    K = np.array([3 * m + g for m in mortar_idx for g in range(3)], dtype=np.int64)   # column order 3 i + gamma
    F = np.setdiff1d(np.arange(N3), K)
    M = np.zeros((N3, 3 * nu))
    M[K, np.arange(3 * nu)] = 1.0
    if F.size:
        # steps 1-3: drop the constrained rows, take the constrained columns as
        # right-hand sides and the free columns as the matrix; step 4: solve
        M[F, :] = -np.linalg.solve(Acc[np.ix_(F, F)], Acc[np.ix_(F, K)])
    return M


def build_mortars(P, mesh, n, beta=4.0, kind="gaussian", A=None):
    """Mortar node indices and the blocks of Q^o for every interface:
    P.H[c] (N_c x nu) for Gaussian mortars (Eq. 8), and P.M[c]
    (3 N_c x 3 nu, rows 3 v + g, columns 3 i + gamma) for both kinds
    (Gaussian: H_c (x) I_3; algebraic: algebraic_block of the interface block
    of A, which must then be given)."""
    P.mortar_idx, P.H, P.M = [], [], []
    P.mortar_kind = kind
    for nodes in P.iface_nodes:
        nu = min(n, len(nodes))
        idx = place_mortars(mesh.xyz[nodes], nu)
        P.mortar_idx.append(idx)
        if kind == "gaussian":
            H = gaussian_weights(mesh.xyz[nodes], idx, beta)
            P.H.append(H)
            P.M.append(np.kron(H, np.eye(3)))
        elif kind == "algebraic":
            d = (3 * np.asarray(nodes, dtype=np.int64)[:, None] + np.arange(3)).ravel()
            P.H.append(None)
            P.M.append(algebraic_block(A[d][:, d], idx))
        else:
            raise ValueError(kind)
    return P
