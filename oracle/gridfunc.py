"""Operator algebra on the CPM discretization (paper Sec. 3.1.2, grid functions:
identity and the Laplace-Beltrami operator of eq. lapBel / eq. semiDisc, added
and composed; Sec. 4.1.2: the shifted biharmonic equation (c + Lap_S^2) u = f).

Sums and compositions of the identity and the second-order Laplace-Beltrami
operator L = Lap_S^h are polynomials in L, P(L) = sum_k a_k L^k; the biharmonic
is L L and the shifted biharmonic c I + L L. With the stabilized operator of the
band, A(c) = c I - L, so L = c I - A(c) for any shift c.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def laplace_beltrami(A: sp.csr_matrix, c: float) -> sp.csr_matrix:
    """L = c I - A(c) from the stabilized operator assembled at shift c."""
    n = A.shape[0]
    return sp.csr_matrix(c * sp.identity(n, format="csr") - A)


def poly_matrix(L: sp.csr_matrix, coef) -> sp.csr_matrix:
    """sum_k coef[k] L^k assembled (Horner: ((a_m L + a_{m-1}) L + ...) )."""
    n = L.shape[0]
    Id = sp.identity(n, format="csr")
    M = coef[-1] * Id
    for a in reversed(coef[:-1]):
        M = sp.csr_matrix(M @ L + a * Id)
    return M


def poly_apply(L: sp.csr_matrix, coef, x: np.ndarray) -> np.ndarray:
    """sum_k coef[k] L^k x by repeated products (no assembled powers)."""
    y = coef[0] * x
    v = x
    for a in coef[1:]:
        v = L @ v
        y = y + a * v
    return y
