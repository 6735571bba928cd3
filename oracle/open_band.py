"""Open surfaces with boundary conditions (paper Sec. 2.1 and Sec. 4.1.6: a
user-defined hemisphere whose circular boundary carries homogeneous Neumann
conditions on one part and homogeneous Dirichlet conditions on the rest).

The surface is given by a closest point function that also reports, for each
closest point on the boundary, whether homogeneous Dirichlet conditions hold
there. Readings (the paper describes the treatment in words and defers the
formulas to the eigenvalue-problem reference it cites):
  * Neumann (natural): a node whose closest point lies on the boundary takes
    the extension u(cp(x)) like any other node;
  * Dirichlet (mirrored): a node x whose closest point c = cp(x) lies on the
    Dirichlet part takes -u(cp(2c - x)), the value at the closest point of its
    mirror image through c, negated (an odd reflection, so that u vanishes on
    the boundary to second order).
Each extension row is therefore `sign * interpolation at ip`, with ip = cp and
sign = +1 for ordinary nodes and ip = cp(2 cp(x) - x), sign = -1 for mirrored
ones. The band follows the closed-surface rules with ip in place of cp:
B_gamma = {x : |x - cp(x)| <= gamma}, Sigma_A = union of the cubes of ip over
B_gamma, Sigma_G = grid neighbours of Sigma_A outside it, closure over
Sigma_A u Sigma_G.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .band import Band, coords, cube_offsets, distance, grid_shape, ijk_of, keys_of, stencil_base
from .operator import bary_weights_1d


def hemisphere(dirichlet=None):
    """Unit upper hemisphere z >= 0 about the origin. Points with z >= 0 project
    radially; points below the plane z = 0 have their closest point on the rim
    circle, (x, y, 0)/|(x, y)|. `dirichlet(phi)` (phi the azimuth of the rim
    point) marks the rim points with Dirichlet conditions (None: all Neumann); the
    flag is set for every point whose closest point is on a marked part of the rim.
    Returns f(x) -> (cp, flag)."""
    def f(x):
        x = np.asarray(x, dtype=np.float64)
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            r = np.sqrt(X * X + Y * Y + Z * Z)
            cap = np.stack([X / r, Y / r, Z / r], axis=1)
            rho = np.sqrt(X * X + Y * Y)
            rim = np.stack([X / rho, Y / rho, np.zeros_like(X)], axis=1)
        below = Z < 0.0
        cp = np.where(below[:, None], rim, cap)
        flag = np.zeros(x.shape[0], dtype=np.int32)
        if dirichlet is not None:
            # a closest point on the rim: every point with z <= 0 (on the plane the radial and
            # the rim projections coincide)
            phi = np.arctan2(cp[:, 1], cp[:, 0])
            flag = ((Z <= 0.0) & np.asarray(dirichlet(phi), dtype=bool)).astype(np.int32)
        return cp, flag
    return f


def interp_points(cpflag, x):
    """(cp, ip, sign) of points x: ip = cp, sign = 1, except ip = cp(2 cp - x), sign = -1
    where the closest point carries Dirichlet conditions."""
    cp, flag = cpflag(x)
    ip = cp.copy()
    sign = np.ones(x.shape[0])
    m = flag != 0
    if m.any():
        xb = 2.0 * cp[m] - x[m]
        cpb, _ = cpflag(xb)
        ip[m] = cpb
        sign[m] = -1.0
    return cp, ip, sign


@dataclass
class OpenBand(Band):
    ip_active: np.ndarray = None
    ip_ghost: np.ndarray = None
    sign_active: np.ndarray = None
    sign_ghost: np.ndarray = None

    @property
    def all_ip(self):
        return np.concatenate([self.ip_active, self.ip_ghost])

    @property
    def all_sign(self):
        return np.concatenate([self.sign_active, self.sign_ghost])


def _cube_keys(ip, lo, h, p, shape):
    b = stencil_base(ip, lo, h, p)
    offs = cube_offsets(ip.shape[1], p)
    pts = (b[:, None, :] + offs[None, :, :]).reshape(-1, ip.shape[1])
    if (pts < 0).any() or (pts >= np.asarray(shape)[None, :]).any():
        raise ValueError("band reaches outside the grid box")
    return keys_of(pts, shape)


def build_open_band(cpflag, d, h, p, lo, hi, gamma) -> OpenBand:
    """B_gamma by brute force over the grid, then Sigma_A, Sigma_G and the closure with
    the mirrored interpolation points."""
    lo = np.asarray(lo, dtype=np.float64)
    shape = grid_shape(lo, hi, h)
    thr = gamma * (1.0 + 1e-10)
    allijk = np.array(list(itertools.product(*[range(s) for s in shape])), dtype=np.int64)
    x = coords(allijk, lo, h)
    cp, flag = cpflag(x)
    inb = distance(x, cp) <= thr
    bkeys = keys_of(allijk[inb], shape)
    _, ipb, _ = interp_points(cpflag, x[inb])
    active = np.unique(_cube_keys(ipb, lo, h, p, shape))
    nbr = np.eye(d, dtype=np.int64)
    iters = 0
    while True:
        aijk = ijk_of(active, shape)
        cand = np.concatenate([keys_of(aijk + s * nbr[k], shape) for k in range(d) for s in (-1, 1)])
        ghost = np.setdiff1d(np.unique(cand), active, assume_unique=True)
        allk = np.concatenate([active, ghost])
        _, ip_all, _ = interp_points(cpflag, coords(ijk_of(allk, shape), lo, h))
        if not np.isfinite(ip_all).all():
            raise ValueError("a band node has no unique closest point; refine h")
        missing = np.setdiff1d(np.unique(_cube_keys(ip_all, lo, h, p, shape)), active, assume_unique=True)
        if missing.size == 0:
            break
        iters += 1
        if iters > 1:
            raise RuntimeError("band closure did not converge")
        active = np.union1d(active, missing)
    ca, ia, sa = interp_points(cpflag, coords(ijk_of(active, shape), lo, h))
    cg, ig, sg = interp_points(cpflag, coords(ijk_of(ghost, shape), lo, h))
    return OpenBand(d=d, p=p, h=h, lo=lo, shape=shape, gamma=gamma, active_keys=active, ghost_keys=ghost,
                    active_ijk=ijk_of(active, shape), ghost_ijk=ijk_of(ghost, shape), cp_active=ca, cp_ghost=cg,
                    n_band=int(bkeys.size), closure_iterations=iters, periodic=(),
                    ip_active=ia, ip_ghost=ig, sign_active=sa, sign_ghost=sg)


def assemble_E_open(band: OpenBand) -> sp.csr_matrix:
    """E with rows sign * (tensor barycentric weights at ip) over the cube of ip."""
    ip = band.all_ip
    d, p = band.d, band.p
    b = stencil_base(ip, band.lo, band.h, p)
    t = (ip - band.lo[None, :]) / band.h - b
    offs = cube_offsets(d, p)
    W = np.ones((ip.shape[0], offs.shape[0]))
    for k in range(d):
        W *= bary_weights_1d(t[:, k], p)[:, offs[:, k]]
    W *= band.all_sign[:, None]
    pts = (b[:, None, :] + offs[None, :, :]).reshape(-1, d)
    cols = np.searchsorted(band.active_keys, keys_of(pts, band.shape))
    if not (band.active_keys[np.minimum(cols, band.active_keys.size - 1)] == keys_of(pts, band.shape)).all():
        raise RuntimeError("node missing from the band (closure violated)")
    rows = np.repeat(np.arange(ip.shape[0]), offs.shape[0])
    E = sp.csr_matrix((W.ravel(), (rows, cols)), shape=(ip.shape[0], band.n_active))
    E.sum_duplicates()
    return E
