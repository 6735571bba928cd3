"""Closest point functions cp_S(x) = argmin_{y in S} |x - y|_2 (paper Sec. 2.1, eq. cpFunc).

Analytic surfaces only: circle and sphere (radial projection), torus
(projection onto the tube's centre circle, then radially within the tube),
ellipsoid (Lagrange-multiplier root, found by bisection), and the straight
line used by the periodic reduction test. All FP64; each formula is written
with an explicit operation order.
"""
from __future__ import annotations

import numpy as np


def cp_sphere(x: np.ndarray, center, R: float) -> np.ndarray:
    """Circle (d=2) or sphere (d=3): cp = c + (R/|x-c|)(x-c)."""
    q = x - np.asarray(center, dtype=np.float64)
    if q.shape[1] == 2:
        n = np.sqrt(q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1])
    else:
        n = np.sqrt(q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1] + q[:, 2] * q[:, 2])
    # the centre itself has no unique closest point; its NaN lies far outside
    # any band and is never used
    with np.errstate(divide="ignore", invalid="ignore"):
        s = R / n
        return np.asarray(center, dtype=np.float64) + s[:, None] * q


def cp_torus(x: np.ndarray, R: float, r: float) -> np.ndarray:
    """Torus about the z axis, major radius R, minor radius r.

    The nearest point of the centre circle is q = (R/rho)(x, y, 0); the closest
    point on the tube is q + (r/|x-q|)(x-q).
    """
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    rho = np.sqrt(X * X + Y * Y)
    sr = R / rho
    qx = sr * X
    qy = sr * Y
    ex = X - qx
    ey = Y - qy
    m = np.sqrt(ex * ex + ey * ey + Z * Z)
    s = r / m
    return np.stack([qx + s * ex, qy + s * ey, s * Z], axis=1)


def cp_ellipsoid(x: np.ndarray, axes) -> np.ndarray:
    """Axis-aligned ellipsoid sum (y_k/a_k)^2 = 1 centred at the origin.

    The closest point is y_k = a_k^2 x_k / (a_k^2 + t) where t is the root of
    F(t) = sum_k (a_k x_k / (a_k^2 + t))^2 - 1, which is strictly decreasing on
    t > -min a_k^2. The root is bracketed by [-amin^2 + amin |x_min|,
    -amin^2 + |(a_k x_k)|] (amin the smallest semi-axis, x_min its coordinate)
    and found by bisection until the midpoint no longer moves.

    A point whose coordinates along every smallest axis vanish and whose
    G = sum over the other axes of (a_k x_k / (a_k^2 - amin^2))^2 is below 1
    has no root above -amin^2: it lies on the medial set, where the closest
    point is not unique (two mirror points). Such points get NaN.
    """
    a = np.asarray(axes, dtype=np.float64)
    a2 = a * a
    kmin = int(np.argmin(a))
    amin = a[kmin]
    ax = x * a[None, :]
    small = a == amin
    on_min_axis = (x[:, small] != 0.0).any(axis=1)
    G = np.zeros(x.shape[0])
    for k in np.flatnonzero(~small):
        rk = ax[:, k] / (a2[k] - a2[kmin])
        G = G + rk * rk
    medial = ~on_min_axis & (G < 1.0)
    nrm = np.sqrt(ax[:, 0] * ax[:, 0] + ax[:, 1] * ax[:, 1] + ax[:, 2] * ax[:, 2])
    lo = -a2[kmin] + amin * np.abs(x[:, kmin])
    hi = -a2[kmin] + nrm
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        r0 = ax[:, 0] / (a2[0] + mid)
        r1 = ax[:, 1] / (a2[1] + mid)
        r2 = ax[:, 2] / (a2[2] + mid)
        F = r0 * r0 + r1 * r1 + r2 * r2 - 1.0
        moved = (mid != lo) & (mid != hi)
        if not moved.any():
            break
        pos = F > 0.0
        lo = np.where(moved & pos, mid, lo)
        hi = np.where(moved & ~pos, mid, hi)
        zero = moved & (F == 0.0)
        lo = np.where(zero, mid, lo)
        hi = np.where(zero, mid, hi)
    t = 0.5 * (lo + hi)
    y = a2[None, :] * x / (a2[None, :] + t[:, None])
    y[medial] = np.nan
    return y


def cp_line(x: np.ndarray, y0: float) -> np.ndarray:
    """Straight line y = y0 in the plane: cp = (x, y0)."""
    out = x.copy()
    out[:, 1] = y0
    return out


def make_cp(kind: str, params):
    """Return cp(x) for a named analytic surface."""
    if kind in ("circle", "sphere"):
        R = params[0]
        center = tuple(params[1:]) if len(params) > 1 else None

        def f(x):
            c = center if center is not None else (0.0,) * x.shape[1]
            return cp_sphere(x, c, R)
        return f
    if kind == "torus":
        return lambda x: cp_torus(x, params[0], params[1])
    if kind == "ellipsoid":
        return lambda x: cp_ellipsoid(x, params)
    if kind == "line":
        return lambda x: cp_line(x, params[0])
    raise ValueError(kind)


def distance(x: np.ndarray, cp: np.ndarray) -> np.ndarray:
    """|x - cp(x)|_2, summed coordinate by coordinate."""
    e = x - cp
    s = e[:, 0] * e[:, 0]
    for k in range(1, x.shape[1]):
        s = s + e[:, k] * e[:, k]
    return np.sqrt(s)
