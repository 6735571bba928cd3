"""Extension E, neighbour sum O and the stabilized CPM operator A (paper Sec. 2.1).

  E   (N_A+N_G) x N_A : row j holds the tensor-product degree-p barycentric
      Lagrange weights (Berrut & Trefethen, "Barycentric Lagrange
      interpolation", SIAM Review 2004) of cp(x_j) on its interpolation cube.
  O   N_A x (N_A+N_G) : (O v)_i = sum over the 2d grid neighbours of x_i.
  Delta_S^h = -(2d/h^2) I + (Delta^h + (2d/h^2) I) E       (eq. lapBel)
            = -(2d/h^2) I + h^-2 O E      (Delta^h + (2d/h^2)I is h^-2 times the neighbour sum)
  A   = c I - Delta_S^h = (c + 2d/h^2) I - h^-2 O E        (eq. shiftPoisson)
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .band import Band, coords, cube_offsets, ijk_of, keys_of, stencil_base, _wrap


def bary_weights_1d(t: np.ndarray, p: int) -> np.ndarray:
    """Barycentric Lagrange basis on equispaced nodes 0..p at points t -> (n, p+1).

    w_j = (-1)^j C(p, j); l_j(t) = (w_j/(t-j)) / sum_k w_k/(t-k); l_j = delta_jk
    when t coincides with node k.
    """
    t = np.asarray(t, dtype=np.float64)
    w = np.array([(-1) ** j * math.comb(p, j) for j in range(p + 1)], dtype=np.float64)
    diff = t[:, None] - np.arange(p + 1, dtype=np.float64)[None, :]
    exact = diff == 0.0
    with np.errstate(divide="ignore", invalid="ignore"):
        q = w[None, :] / diff
        out = q / q.sum(axis=1, keepdims=True)
    hit = exact.any(axis=1)
    out[hit] = exact[hit].astype(np.float64)
    return out


def extension_rows(cp: np.ndarray, lo, h, p):
    """Cube lower corners b (n,d) and the (n,(p+1)^d) tensor weights, cube in cube_offsets order."""
    d = cp.shape[1]
    b = stencil_base(cp, lo, h, p)
    t = (cp - np.asarray(lo, dtype=np.float64)[None, :]) / h - b
    l1 = [bary_weights_1d(t[:, k], p) for k in range(d)]
    offs = cube_offsets(d, p)
    W = np.ones((cp.shape[0], offs.shape[0]))
    for k in range(d):
        W *= l1[k][:, offs[:, k]]
    return b, W


def _lookup(sorted_keys: np.ndarray, keys: np.ndarray) -> np.ndarray:
    pos = np.searchsorted(sorted_keys, keys)
    pos = np.minimum(pos, sorted_keys.size - 1)
    if not (sorted_keys[pos] == keys).all():
        raise RuntimeError("node missing from the band (closure violated)")
    return pos


def assemble_E(band: Band) -> sp.csr_matrix:
    """E as CSR, rows = Sigma_A then Sigma_G (each by ascending key), columns = Sigma_A."""
    cp = band.all_cp
    b, W = extension_rows(cp, band.lo, band.h, band.p)
    offs = cube_offsets(band.d, band.p)
    pts = (b[:, None, :] + offs[None, :, :]).reshape(-1, band.d)
    cols = _lookup(band.active_keys, keys_of(_wrap(pts, band.shape, band.periodic), band.shape))
    n = cp.shape[0]
    rows = np.repeat(np.arange(n), offs.shape[0])
    E = sp.csr_matrix((W.ravel(), (rows, cols)), shape=(n, band.n_active))
    E.sum_duplicates()
    return E


def assemble_O(band: Band) -> sp.csr_matrix:
    """Neighbour-sum matrix: row i (active) has a 1 at each of its 2d grid neighbours."""
    allk = band.all_keys
    order = np.argsort(allk)
    sk = allk[order]
    d = band.d
    rows, cols = [], []
    for k in range(d):
        for s in (-1, 1):
            nb = band.active_ijk.copy()
            nb[:, k] += s
            key = keys_of(_wrap(nb, band.shape, band.periodic), band.shape)
            cols.append(order[_lookup(sk, key)])
            rows.append(np.arange(band.n_active))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    return sp.csr_matrix((np.ones(rows.size), (rows, cols)),
                         shape=(band.n_active, band.n_active + band.n_ghost))


def assemble_A(band: Band, c: float, E=None, O=None) -> sp.csr_matrix:
    """A = (c + 2d/h^2) I - h^-2 O E on Sigma_A."""
    E = assemble_E(band) if E is None else E
    O = assemble_O(band) if O is None else O
    h2 = band.h * band.h
    A = (c + 2.0 * band.d / h2) * sp.identity(band.n_active, format="csr") - (O @ E) / h2
    return sp.csr_matrix(A)


def structural_pattern(band: Band, O=None) -> sp.csr_matrix:
    """Structural nonzero pattern of A: diagonal plus every cube node of every neighbour
    (exactly-zero interpolation weights included), as a 0/1 CSR matrix."""
    O = assemble_O(band) if O is None else O
    # built from the cubes themselves so that exactly-zero weights keep their entry
    cp = band.all_cp
    b = stencil_base(cp, band.lo, band.h, band.p)
    offs = cube_offsets(band.d, band.p)
    pts = (b[:, None, :] + offs[None, :, :]).reshape(-1, band.d)
    cols = _lookup(band.active_keys, keys_of(_wrap(pts, band.shape, band.periodic), band.shape))
    n = cp.shape[0]
    Es = sp.csr_matrix((np.ones(cols.size), (np.repeat(np.arange(n), offs.shape[0]), cols)),
                       shape=(n, band.n_active))
    P = (O @ Es) + sp.identity(band.n_active, format="csr")
    P = sp.csr_matrix(P)
    P.data[:] = 1.0
    return P


def values_on_pattern(A: sp.csr_matrix, P: sp.csr_matrix) -> sp.csr_matrix:
    """Matrix with the nonzero structure of P and the values of A (zero where A has none)."""
    A = sp.csr_matrix(A)
    P = sp.csr_matrix(P)
    P.sort_indices()
    n = A.shape[1]
    ak = np.repeat(np.arange(A.shape[0], dtype=np.int64), np.diff(A.indptr)) * n + A.indices
    order = np.argsort(ak)
    ak = ak[order]
    av = A.data[order]
    pk = np.repeat(np.arange(P.shape[0], dtype=np.int64), np.diff(P.indptr)) * n + P.indices
    pos = np.minimum(np.searchsorted(ak, pk), max(ak.size - 1, 0))
    hit = ak[pos] == pk if ak.size else np.zeros(pk.size, dtype=bool)
    vals = np.where(hit, av[pos] if ak.size else 0.0, 0.0)
    if hit.sum() != A.nnz:
        raise RuntimeError("A has entries outside the structural pattern")
    return sp.csr_matrix((vals, P.indices.copy(), P.indptr.copy()), shape=P.shape)


def apply_rows(cpfun, d: int, p: int, h: float, lo, shape, c: float, row_keys, u_keys, u_vals,
               chunk: int = 20000, magnitude: bool = False) -> np.ndarray:
    """(A u)_i = (c + 2d/h^2) u_i - h^-2 sum_{n in N(i)} (E u)_n for the grid nodes with
    keys row_keys, straight from the definitions (eq. lapBel) without assembling A:
    each neighbour's closest point cp(x_n) is evaluated by `cpfun`, its cube and
    barycentric weights come from extension_rows, and u is read at the cube nodes.

    u is given as values u_vals [(N, R) or (N,)] at the sorted grid keys u_keys (the
    active nodes); a cube node missing from u_keys raises (the band was not closed).
    Rows are processed `chunk` at a time. Returns an array shaped like u_vals[row].
    magnitude=True returns instead the sum of the magnitudes of the terms,
    (c + 2d/h^2)|u_i| + h^-2 sum_n sum_alpha |w_alpha| |u|, the forward-error
    scale of row i for any summation order.
    """
    row_keys = np.asarray(row_keys, dtype=np.int64)
    u_keys = np.asarray(u_keys, dtype=np.int64)
    uv = np.asarray(u_vals, dtype=np.float64)
    if magnitude:
        uv = np.abs(uv)
    one = uv.ndim == 1
    uv = uv.reshape(uv.shape[0], -1)
    if np.any(np.diff(u_keys) <= 0):
        raise ValueError("u_keys must be strictly increasing")
    lo = np.asarray(lo, dtype=np.float64)
    offs = cube_offsets(d, p)
    h2 = h * h
    ntot = int(np.prod(np.asarray(shape, dtype=np.int64)))
    if ntot <= 100_000_000:   # dense key -> position map
        where = np.full(ntot, -1, dtype=np.int64)
        where[u_keys] = np.arange(u_keys.size)

        def find(keys):
            pos = where[keys]
            if (pos < 0).any():
                raise RuntimeError("node missing from the band (closure violated)")
            return pos
    else:
        def find(keys):
            return _lookup(u_keys, keys)

    out = np.empty((row_keys.size, uv.shape[1]))
    for s in range(0, row_keys.size, chunk):
        rk = row_keys[s:s + chunk]
        ijk = ijk_of(rk, shape)
        acc = np.zeros((rk.size, uv.shape[1]))
        for k in range(d):
            for sg in (-1, 1):
                nb = ijk.copy()
                nb[:, k] += sg
                b, W = extension_rows(cpfun(coords(nb, lo, h)), lo, h, p)
                if magnitude:
                    W = np.abs(W)
                pts = (b[:, None, :] + offs[None, :, :]).reshape(-1, d)
                if (pts < 0).any() or (pts >= np.asarray(shape)[None, :]).any():
                    raise RuntimeError("interpolation cube leaves the grid")
                vals = uv[find(keys_of(pts, shape))].reshape(rk.size, offs.shape[0], uv.shape[1])
                acc += np.einsum("nq,nqr->nr", W, vals)
        out[s:s + rk.size] = (c + 2.0 * d / h2) * uv[find(rk)] + (acc if magnitude else -acc) / h2
    return out[:, 0] if one else out
