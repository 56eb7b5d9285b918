"""Oracle: right-preconditioned GMRES and flexible GMRES.  TEST
INFRASTRUCTURE ONLY.

The paper solves A x = b with right-preconditioned GMRES and stops when the
normalised residual |A x - b| / |b| falls below a tolerance or after 300
iterations (Sec. 5).

Reading R10 (the paper does not state restart, start vector, orthogonalisation
or when the true residual is checked): x0 = 0 unless given, restart m = 50,
modified Gram-Schmidt Arnoldi, Givens rotations for the least-squares
problem; whenever the Arnoldi residual estimate drops below the tolerance,
and at the end of every cycle, x is formed and the *true* residual is
computed; the solve stops when that is below the tolerance, otherwise a new
cycle starts from the current x.  ``flexible=True`` stores z_j = M^-1 v_j and
forms x = x0 + Z y (flexible GMRES), which equals GMRES for a fixed M.
"""
from __future__ import annotations

import numpy as np


class Result:
    pass


def gmres(A, b, apply_M, x0=None, tol=1e-8, restart=50, maxit=300, flexible=False,
          max_steps=None):
    """Returns a Result with x, iters, converged, rel_res (true), history
    (Arnoldi estimates per step) and true_history (at every check).

    max_steps: if given, stop after exactly that many Arnoldi steps (forming x)
    regardless of convergence.
    """
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=float)
    bnorm = np.linalg.norm(b)
    res = Result()
    res.history, res.true_history = [], []
    if bnorm == 0.0:
        res.x, res.iters, res.converged, res.rel_res = np.zeros(n), 0, True, 0.0
        return res
    it = 0
    limit = maxit if max_steps is None else max_steps
    converged = False
    rel_true = np.linalg.norm(b - A @ x) / bnorm
    res.true_history.append(rel_true)
    if rel_true < tol and max_steps is None:
        converged = True
    while not converged and it < limit:
        r = b - A @ x
        beta = np.linalg.norm(r)
        m = restart
        V = np.zeros((n, m + 1))
        Z = np.zeros((n, m)) if flexible else None
        Hm = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        j_done = 0
        stop_cycle = False
        for j in range(m):
            zj = apply_M(V[:, j])
            if flexible:
                Z[:, j] = zj
            w = A @ zj
            for i in range(j + 1):                      # modified Gram-Schmidt
                Hm[i, j] = np.dot(w, V[:, i])
                w = w - Hm[i, j] * V[:, i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] != 0.0:
                V[:, j + 1] = w / Hm[j + 1, j]
            for i in range(j):                          # previous rotations
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            d = np.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j], sn[j] = Hm[j, j] / d, Hm[j + 1, j] / d
            Hm[j, j] = d
            Hm[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            est = abs(g[j + 1]) / bnorm
            res.history.append(est)
            if it >= limit or (max_steps is None and est < tol):
                stop_cycle = True
                break
        k = j_done
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):                  # back substitution
            y[i] = (g[i] - Hm[i, i + 1:k] @ y[i + 1:k]) / Hm[i, i]
        if flexible:
            x = x + Z[:, :k] @ y
        else:
            x = x + apply_M(V[:, :k] @ y)
        rel_true = np.linalg.norm(b - A @ x) / bnorm
        res.true_history.append(rel_true)
        if max_steps is None and rel_true < tol:
            converged = True
        del stop_cycle
    res.x, res.iters, res.converged, res.rel_res = x, it, converged, rel_true
    return res
