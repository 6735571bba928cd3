"""Fourth-order Laplace-Beltrami grid function of the closest point method
(paper Sec. 3.1.2: the built-in grid functions include second- and fourth-order
accurate Laplace-Beltrami operators).

Test infrastructure only (the oracle): plain NumPy/SciPy FP64.

Along each axis the fourth-order centred second difference of the extended
function v = E u is (-v_{i-2} + 16 v_{i-1} - 30 v_i + 16 v_{i+1} - v_{i+2}) / (12 h^2).
In the stabilized form of eq. lapBel the node's own term uses u_i instead of
its extension v_i:
    Lap4 u_i = -(30 d / (12 h^2)) u_i
               + (1 / (12 h^2)) sum_k [16 (v_{i+e_k} + v_{i-e_k}) - (v_{i+2e_k} + v_{i-2e_k})]
    A4(c) = c I - Lap4 = (c + 30d/(12h^2)) I - (1/(12h^2)) (16 O1 - O2) E
with O1 the sum over the 2d nearest grid neighbours and O2 over the 2d nodes two
steps away along an axis. The stencil reaches two nodes, so the ghost set holds
every grid node within two steps along an axis of Sigma_A that is not in Sigma_A,
and the band radius grows by one h along the normal-most axis:
    gamma = h sqrt((d-1)((p+1)/2)^2 + (2 + (p+1)/2)^2).
With degree-p interpolation the method's error is O(h^4) + O(h^{p+1} / h^2): p = 5
gives fourth order, p = 3 second order.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .band import Band, _cubes, _wrap, build_band, coords, ijk_of, keys_of
from .operator import _lookup, assemble_E


def gamma_reach(d: int, p: int, h: float, reach: int) -> float:
    """Band radius whose cube-and-stencil box holds the stencil's reach (reach = 1: the
    Ruuth-Merriman radius)."""
    a = (p + 1) / 2.0
    return h * math.sqrt((d - 1) * a * a + (reach + a) ** 2)


def build_band_reach(cpfun, d, h, p, lo, hi, reach=2, gamma=None, periodic=()) -> Band:
    """The band of build_band with a ghost set of every node within `reach` steps along
    an axis of Sigma_A; closure (cubes of all ghosts inside Sigma_A) checked again, with
    at most one growth step."""
    gamma = gamma_reach(d, p, h, reach) if gamma is None else gamma
    b1 = build_band(cpfun, d, h, p, lo, hi, gamma, periodic=periodic)
    shape, lo = b1.shape, b1.lo
    active = b1.active_keys
    nbr = np.eye(d, dtype=np.int64)
    iters = 0
    while True:
        aijk = ijk_of(active, shape)
        cand = np.concatenate([keys_of(_wrap(aijk + s * nbr[k], shape, periodic), shape)
                               for k in range(d) for s in range(-reach, reach + 1) if s != 0])
        ghost = np.setdiff1d(np.unique(cand), active, assume_unique=True)
        cpg = cpfun(coords(ijk_of(ghost, shape), lo, h))
        if not np.isfinite(cpg).all():
            raise ValueError("a band node has no unique closest point; refine h")
        missing = np.setdiff1d(np.unique(_cubes(cpg, lo, h, p, shape, periodic)), active, assume_unique=True)
        if missing.size == 0:
            break
        iters += 1
        if iters > 1:
            raise RuntimeError("band closure did not converge")
        active = np.union1d(active, missing)
    cpa = cpfun(coords(ijk_of(active, shape), lo, h))
    return Band(d=d, p=p, h=h, lo=lo, shape=shape, gamma=gamma, active_keys=active, ghost_keys=ghost,
                active_ijk=ijk_of(active, shape), ghost_ijk=ijk_of(ghost, shape), cp_active=cpa,
                cp_ghost=cpg, n_band=b1.n_band, closure_iterations=b1.closure_iterations + iters,
                periodic=tuple(periodic))


def assemble_O_step(band: Band, step: int) -> sp.csr_matrix:
    """(O_s v)_i = sum of v over the 2d grid nodes i +- s e_k (rows: Sigma_A)."""
    allk = band.all_keys
    order = np.argsort(allk)
    sk = allk[order]
    rows, cols = [], []
    for k in range(band.d):
        for s in (-step, step):
            nb = band.active_ijk.copy()
            nb[:, k] += s
            key = keys_of(_wrap(nb, band.shape, band.periodic), band.shape)
            cols.append(order[_lookup(sk, key)])
            rows.append(np.arange(band.n_active))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(band.n_active, band.n_active + band.n_ghost))


def assemble_A4(band: Band, c: float, E=None) -> sp.csr_matrix:
    """A4(c) = (c + 30d/(12h^2)) I - (1/(12h^2)) (16 O1 - O2) E on Sigma_A."""
    E = assemble_E(band) if E is None else E
    O1 = assemble_O_step(band, 1)
    O2 = assemble_O_step(band, 2)
    s = 12.0 * band.h * band.h
    n = band.n_active
    A = (c + 30.0 * band.d / s) * sp.identity(n, format="csr") - ((16.0 * O1 - O2) @ E) / s
    return sp.csr_matrix(A)

