"""User-defined surfaces for cpm.Band.from_closest_point (callback closest points).

Each factory returns fn(x) -> (cp, flag) over an (n, d) array of points: the
closest points and, for open surfaces, flag = 1 where the closest point lies on
a boundary part with homogeneous Dirichlet conditions (the library mirrors those
extension rows), 0 elsewhere (interior, or natural Neumann boundary).
"""
from __future__ import annotations

import numpy as np


def hemisphere(radius: float = 1.0, dirichlet=None):
    """Upper hemisphere z >= 0 of the sphere of the given radius about the origin (the
    user-defined open surface of the paper's Schnackenberg example). Points with z >= 0
    project radially onto the cap; points below the plane z = 0 are closest to the rim
    circle, at radius * (x, y, 0)/|(x, y)|. dirichlet(phi) -> bool array, phi the azimuth
    of the rim point, marks Dirichlet parts of the rim (None: natural Neumann on all of
    it; for the paper's example use lambda phi: np.sin(3 * phi) < -0.5)."""
    R = float(radius)

    def fn(x):
        x = np.asarray(x, dtype=np.float64)
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        on_cap = Z >= 0.0
        cp = np.empty_like(x)
        with np.errstate(divide="ignore", invalid="ignore"):   # the origin and the z axis below: no unique cp
            s = R / np.sqrt(X * X + Y * Y + Z * Z)
            t = R / np.sqrt(X * X + Y * Y)
            cp[:, 0] = np.where(on_cap, X * s, X * t)
            cp[:, 1] = np.where(on_cap, Y * s, Y * t)
            cp[:, 2] = np.where(on_cap, Z * s, 0.0)
        flag = np.zeros(x.shape[0], dtype=np.int32)
        if dirichlet is not None:
            phi = np.arctan2(cp[:, 1], cp[:, 0])
            flag[(Z <= 0.0) & np.asarray(dirichlet(phi), dtype=bool)] = 1
        return cp, flag
    return fn
