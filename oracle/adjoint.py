"""Adjoint of the CPM solve (the transpose of the paper's operator, Sec. 2.1, eq. lapBel).

For u = A(c)^-1 f with A(c) = c I + K (K = (2d/h^2) I - h^-2 O E independent of c)
and a loss L(u):
    A^T lambda = dL/du,   dL/df = lambda,   dL/dc = -lambda . u
(differentiate A u = f: A du = df - dc u). Here L = |u - u_t|_2^2, dL/du = 2(u - u_t).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def transpose_apply(A: sp.csr_matrix, y: np.ndarray) -> np.ndarray:
    return A.T @ y


def quadratic_loss_grads(A: sp.csr_matrix, f: np.ndarray, u_target: np.ndarray, dense=False):
    """Returns (L, u, dL/df, dL/dc) by a direct solve of A u = f and A^T lambda = 2(u - u_t)."""
    if dense:
        Ad = A.toarray()
        u = np.linalg.solve(Ad, f)
        lam = np.linalg.solve(Ad.T, 2.0 * (u - u_target))
    else:
        lu = spla.splu(sp.csc_matrix(A))
        u = lu.solve(f)
        lam = lu.solve(2.0 * (u - u_target), trans="T")
    L = float(np.dot(u - u_target, u - u_target))
    return L, u, lam, -float(np.dot(lam, u))
