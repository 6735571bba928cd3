"""Restarted, right-preconditioned flexible GMRES (the paper's default Krylov method,
Sec. 4.1.1 names GMRES as the default solver).

Textbook form (Saad, "Iterative Methods for Sparse Linear Systems", 2nd ed.,
Alg. 9.6 FGMRES): modified Gram-Schmidt Arnoldi on z_j = M^-1 v_j, Givens
rotations on the Hessenberg matrix, x += Z y at the end of each cycle.
Conventions (the paper states none): restart 30, x0 = 0, stop when the true
residual |f - A x|_2 <= rtol |f|_2, checked at every restart; within a cycle
the Givens residual estimate ends the cycle early.
"""
from __future__ import annotations

import numpy as np


def fgmres(A, f, M=None, restart=30, rtol=1e-10, max_it=10000, x0=None):
    """Solve A x = f. A and M are callables (or objects with @). Returns (x, info).

    info = dict(iters, restarts, relres, converged, history).
    """
    matvec = A if callable(A) else (lambda v: A @ v)
    prec = (lambda v: v) if M is None else (M if callable(M) else (lambda v: M @ v))
    n = f.size
    x = np.zeros(n) if x0 is None else x0.astype(np.float64).copy()
    fn = np.linalg.norm(f)
    target = rtol * fn
    it = 0
    hist = []
    restarts = 0
    r = f - matvec(x)
    beta = np.linalg.norm(r)
    hist.append(beta / fn if fn > 0 else 0.0)
    while beta > target and it < max_it:
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = prec(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            if abs(g[j + 1]) <= target or it >= max_it or H[j, j] == 0.0:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        r = f - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta / fn if fn > 0 else 0.0)
        restarts += 1
    return x, dict(iters=it, restarts=restarts, relres=beta / fn if fn > 0 else 0.0,
                   converged=bool(beta <= target), history=hist)
