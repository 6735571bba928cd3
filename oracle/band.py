"""Computational band of the closest point method (paper Sec. 2.1).

Definitions followed (the paper gives the properties, this module the sets):
  * grid nodes x_i = lo + i h, i in {0..n-1}^d;
  * B_gamma  = nodes with |x - cp(x)| <= gamma (1 + 1e-10) (inclusive radius);
  * Sigma_A  = union over x in B_gamma of the (p+1)^d interpolation cube of cp(x)
               (Sec. 2.1: the active set must hold every cube the extension
               reads);
  * Sigma_G  = grid neighbours (+-e_k) of Sigma_A that are not in Sigma_A
               (Sec. 2.1: the ghost set completes the finite-difference
               stencils of the active nodes);
  * closure  = every node of Sigma_A u Sigma_G has its cube inside Sigma_A
               (the extension is evaluated at all of them); a closure loop
               adds missing cube nodes, at most once, else raises.
The interpolation cube of a point c has lower corner
  b = floor((c - lo)/h - (p-1)/2)       (IEEE division, then subtraction)
and nodes b + {0..p}^d.
Nodes are identified by row-major linear keys (first axis slowest); the
oracle orders Sigma_A and Sigma_G by ascending key.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from .surfaces import distance


@dataclass
class Band:
    d: int
    p: int
    h: float
    lo: np.ndarray          # (d,)
    shape: tuple            # grid points per axis
    gamma: float
    active_keys: np.ndarray  # (N_A,) sorted int64
    ghost_keys: np.ndarray   # (N_G,) sorted int64
    active_ijk: np.ndarray   # (N_A, d) int64
    ghost_ijk: np.ndarray    # (N_G, d)
    cp_active: np.ndarray    # (N_A, d)
    cp_ghost: np.ndarray     # (N_G, d)
    n_band: int              # |B_gamma|
    closure_iterations: int
    periodic: tuple = ()

    @property
    def n_active(self):
        return self.active_keys.size

    @property
    def n_ghost(self):
        return self.ghost_keys.size

    @property
    def all_keys(self):
        return np.concatenate([self.active_keys, self.ghost_keys])

    @property
    def all_ijk(self):
        return np.concatenate([self.active_ijk, self.ghost_ijk])

    @property
    def all_cp(self):
        return np.concatenate([self.cp_active, self.cp_ghost])


def grid_shape(lo, hi, h):
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return tuple(int(np.floor((hi[k] - lo[k]) / h + 0.5)) + 1 for k in range(lo.size))


def keys_of(ijk: np.ndarray, shape) -> np.ndarray:
    key = np.zeros(ijk.shape[0], dtype=np.int64)
    for k in range(ijk.shape[1]):
        key = key * int(shape[k]) + ijk[:, k]
    return key


def ijk_of(keys: np.ndarray, shape) -> np.ndarray:
    keys = np.asarray(keys, dtype=np.int64).copy()
    d = len(shape)
    out = np.zeros((keys.size, d), dtype=np.int64)
    for k in range(d - 1, -1, -1):
        out[:, k] = keys % shape[k]
        keys //= shape[k]
    return out


def coords(ijk: np.ndarray, lo, h) -> np.ndarray:
    return np.asarray(lo, dtype=np.float64)[None, :] + ijk.astype(np.float64) * h


def stencil_base(cp: np.ndarray, lo, h, p) -> np.ndarray:
    """Lower corner b = floor((cp - lo)/h - (p-1)/2) of the interpolation cube."""
    t = (cp - np.asarray(lo, dtype=np.float64)[None, :]) / h
    return np.floor(t - (p - 1) / 2.0).astype(np.int64)


def cube_offsets(d, p):
    return np.array(list(itertools.product(range(p + 1), repeat=d)), dtype=np.int64)


def _wrap(ijk, shape, periodic):
    out = ijk.copy()
    for k in range(ijk.shape[1]):
        if k < len(periodic) and periodic[k]:
            out[:, k] %= shape[k]
        elif (out[:, k] < 0).any() or (out[:, k] >= shape[k]).any():
            raise ValueError("band reaches outside the grid box")
    return out


def _cubes(cp, lo, h, p, shape, periodic):
    """All keys of the interpolation cubes of points cp (with repetition)."""
    b = stencil_base(cp, lo, h, p)
    offs = cube_offsets(cp.shape[1], p)
    pts = (b[:, None, :] + offs[None, :, :]).reshape(-1, cp.shape[1])
    return keys_of(_wrap(pts, shape, periodic), shape)


def build_band(cpfun, d, h, p, lo, hi, gamma, periodic=(), prefilter=None,
               chunk_nodes=2_000_000) -> Band:
    """Enumerate B_gamma by brute force over the grid, then Sigma_A, Sigma_G, closure.

    `prefilter(x)` may return a boolean mask of nodes that can possibly lie in
    the band (a lower bound on the distance); it only saves time.
    """
    lo = np.asarray(lo, dtype=np.float64)
    shape = grid_shape(lo, hi, h)
    thr = gamma * (1.0 + 1e-10)
    # ---- B_gamma by brute force, slab by slab over the first axis
    plane = int(np.prod(shape[1:]))
    per = max(1, chunk_nodes // plane)
    band_keys, band_cp = [], []
    rest = np.array(list(itertools.product(*[range(s) for s in shape[1:]])), dtype=np.int64) \
        if d > 1 else np.zeros((1, 0), dtype=np.int64)
    for i0 in range(0, shape[0], per):
        i1 = min(shape[0], i0 + per)
        first = np.repeat(np.arange(i0, i1, dtype=np.int64), rest.shape[0])
        ijk = np.concatenate([first[:, None], np.tile(rest, (i1 - i0, 1))], axis=1)
        x = coords(ijk, lo, h)
        if prefilter is not None:
            m = prefilter(x)
            ijk, x = ijk[m], x[m]
        if ijk.shape[0] == 0:
            continue
        cp = cpfun(x)
        m = distance(x, cp) <= thr
        band_keys.append(keys_of(ijk[m], shape))
        band_cp.append(cp[m])
    bkeys = np.concatenate(band_keys)
    bcp = np.concatenate(band_cp)
    n_band = bkeys.size

    def cp_of(keys):
        pos = np.searchsorted(bkeys, keys)
        pos = np.minimum(pos, bkeys.size - 1)
        hit = bkeys[pos] == keys
        out = np.empty((keys.size, d))
        out[hit] = bcp[pos[hit]]
        if (~hit).any():
            out[~hit] = cpfun(coords(ijk_of(keys[~hit], shape), lo, h))
        return out, hit

    # ---- Sigma_A: union of interpolation cubes of the band's closest points
    active = np.unique(np.concatenate(
        [np.unique(_cubes(bcp[s:s + 100_000], lo, h, p, shape, periodic))
         for s in range(0, n_band, 100_000)]))
    nbr = np.eye(d, dtype=np.int64)
    iters = 0
    while True:
        aijk = ijk_of(active, shape)
        cand = np.concatenate([keys_of(_wrap(aijk + s * nbr[k], shape, periodic), shape)
                               for k in range(d) for s in (-1, 1)])
        ghost = np.setdiff1d(np.unique(cand), active, assume_unique=True)
        allk = np.concatenate([active, ghost])
        cps, _ = cp_of(allk)
        if not np.isfinite(cps).all():
            # a node of Sigma_A u Sigma_G on the medial axis: cp is not unique (Sec. 2.1
            # assumes h small enough that the band stays clear of it)
            raise ValueError("a band node has no unique closest point; refine h")
        need = np.unique(_cubes(cps, lo, h, p, shape, periodic))
        missing = np.setdiff1d(need, active, assume_unique=True)
        if missing.size == 0:
            break
        iters += 1
        if iters > 1:
            raise RuntimeError("band closure did not converge")
        active = np.union1d(active, missing)
    cpa, _ = cp_of(active)
    cpg, _ = cp_of(ghost)
    return Band(d=d, p=p, h=h, lo=lo, shape=shape, gamma=gamma,
                active_keys=active, ghost_keys=ghost,
                active_ijk=ijk_of(active, shape), ghost_ijk=ijk_of(ghost, shape),
                cp_active=cpa, cp_ghost=cpg, n_band=n_band,
                closure_iterations=iters, periodic=tuple(periodic))


def ellipsoid_prefilter(axes, gamma):
    """Nodes with amin |(|x/a|) - 1| > gamma cannot be in the band (x -> x/a is 1/amin-Lipschitz)."""
    a = np.asarray(axes, dtype=np.float64)
    amin = a.min()

    def f(x):
        q = np.sqrt(((x / a[None, :]) ** 2).sum(axis=1))
        return amin * np.abs(q - 1.0) <= gamma * (1.0 + 1e-6) + 1e-12
    return f
