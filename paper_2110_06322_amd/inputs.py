"""Seeded synthetic inputs shared by the library's callers, the tests and the bench.

This module holds no arithmetic of the closest point method itself: it only
turns seeds, grid indices and surface points into numbers (right-hand sides,
target fields, initial conditions, random test vectors, instance parameters).
Both the HIP path and the CPU oracle receive their inputs from here, each
evaluating the same definitions at its own nodes, so that neither side ever
takes an input from the other.

Per-node random values come from a counter-based generator (SplitMix64,
Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014) keyed by (seed, stream, linear grid index): a node's value does
not depend on how either side orders its nodes.
"""
from __future__ import annotations

import math

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def _splitmix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser applied elementwise to uint64 counters."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def _counter(seed: int, stream: int, key: np.ndarray) -> np.ndarray:
    key = np.asarray(key, dtype=np.int64).astype(np.uint64)
    s = _splitmix64(np.uint64((seed * 1_000_003 + stream) & 0xFFFFFFFFFFFFFFFF))
    with np.errstate(over="ignore"):
        return _splitmix64(key * np.uint64(0xD1B54A32D192ED03) ^ s)


def uniform(seed: int, stream: int, key) -> np.ndarray:
    """U[0,1) per key: the top 53 bits of one SplitMix64 draw."""
    r = _counter(seed, stream, key)
    return (r >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normal(seed: int, stream: int, key) -> np.ndarray:
    """N(0,1) per key by Box-Muller on two independent counter draws."""
    key = np.asarray(key, dtype=np.int64)
    u1 = uniform(seed, 2 * stream, key)
    u2 = uniform(seed, 2 * stream + 1, key)
    u1 = 1.0 - u1  # (0, 1]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def linear_key(gidx: np.ndarray, shape) -> np.ndarray:
    """Row-major linear grid index (first axis slowest) of integer grid coordinates."""
    gidx = np.asarray(gidx, dtype=np.int64)
    key = np.zeros(gidx.shape[0], dtype=np.int64)
    for k in range(gidx.shape[1]):
        key = key * int(shape[k]) + gidx[:, k]
    return key


# --------------------------------------------------------------------------
# Surface fields used as right-hand sides / exact solutions / targets
# --------------------------------------------------------------------------

def quartic_harmonics(x: np.ndarray) -> np.ndarray:
    """The nine real solid harmonics of degree 4 at points x (n x 3), columns m=-4..4.

    Homogeneous harmonic polynomials; restricted to the unit sphere they are
    eigenfunctions of the Laplace-Beltrami operator with eigenvalue -l(l+1) = -20.
    """
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    r2 = X * X + Y * Y + Z * Z
    cols = [
        X * Y * (X * X - Y * Y),                     # m = -4
        Y * Z * (3.0 * X * X - Y * Y),               # m = -3
        X * Y * (7.0 * Z * Z - r2),                  # m = -2
        Y * Z * (7.0 * Z * Z - 3.0 * r2),            # m = -1
        35.0 * Z ** 4 - 30.0 * Z * Z * r2 + 3.0 * r2 * r2,  # m = 0
        X * Z * (7.0 * Z * Z - 3.0 * r2),            # m = 1
        (X * X - Y * Y) * (7.0 * Z * Z - r2),        # m = 2
        X * Z * (X * X - 3.0 * Y * Y),               # m = 3
        X ** 4 - 6.0 * X * X * Y * Y + Y ** 4,       # m = 4
    ]
    return np.stack(cols, axis=1)


def sphere_harmonic_coeffs(seed: int) -> np.ndarray:
    """Seeded N(0,1) coefficients a_m, m=-4..4, of a degree-4 spherical harmonic."""
    return np.random.default_rng(seed).standard_normal(9)


def sphere_y4(cp: np.ndarray, seed: int, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Y(cp) = sum_m a_m Y_4^m(n), n = (cp - center)/|cp - center| on a sphere."""
    q = np.asarray(cp, dtype=np.float64) - np.asarray(center, dtype=np.float64)
    n = q / np.sqrt((q * q).sum(axis=1))[:, None]
    return quartic_harmonics(n) @ sphere_harmonic_coeffs(seed)


def circle_sin(cp: np.ndarray, center=(0.0, 0.0)) -> np.ndarray:
    """sin(theta) of a point on a circle about `center`."""
    q = np.asarray(cp, dtype=np.float64) - np.asarray(center, dtype=np.float64)
    return q[:, 1] / np.sqrt((q * q).sum(axis=1))


def torus_angles(cp: np.ndarray, R: float):
    """Toroidal angle phi = atan2(y,x) and poloidal angle theta = atan2(z, rho-R)."""
    x, y, z = cp[:, 0], cp[:, 1], cp[:, 2]
    rho = np.sqrt(x * x + y * y)
    return np.arctan2(y, x), np.arctan2(z, rho - R)


def torus_modes(cp: np.ndarray, R: float, seed: int, nmax: int = 3) -> np.ndarray:
    """sum_{m,n<=nmax} (a_mn cos(m phi + n theta) + b_mn sin(m phi + n theta)) / (1+m^2+n^2)."""
    phi, th = torus_angles(cp, R)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((nmax + 1, nmax + 1))
    b = rng.standard_normal((nmax + 1, nmax + 1))
    out = np.zeros(cp.shape[0])
    for m in range(nmax + 1):
        for n in range(nmax + 1):
            arg = m * phi + n * th
            out += (a[m, n] * np.cos(arg) + b[m, n] * np.sin(arg)) / (1.0 + m * m + n * n)
    return out


def gray_scott_ic(keys: np.ndarray, seed: int):
    """u = 1 - 0.5 xi, v = 0.25 xi', xi, xi' ~ U[0,1) i.i.d. per node."""
    xi = uniform(seed, 11, keys)
    xi2 = uniform(seed, 12, keys)
    return 1.0 - 0.5 * xi, 0.25 * xi2


def batch_instances(seed: int = 3, n_each: int = 16, hs=(0.04, 0.02, 0.01)):
    """The 48-surface batched workload: spheres, ellipsoids, tori at cyclic h.

    Returns a list of dicts {kind, params, h, c, n_rhs}; ellipsoid semi-axes
    ~ U[0.6,1.4]^3, torus minor radius ~ U[0.3,0.5] (major 1), c ~ U[0.5,10]
    per surface, h assigned cyclically by instance index.
    """
    rng = np.random.default_rng(seed)
    out = []
    kinds = ["sphere"] * n_each + ["ellipsoid"] * n_each + ["torus"] * n_each
    for i, kind in enumerate(kinds):
        if kind == "sphere":
            params = (1.0,)
        elif kind == "ellipsoid":
            params = tuple(float(v) for v in rng.uniform(0.6, 1.4, size=3))
        else:
            params = (1.0, float(rng.uniform(0.3, 0.5)))
        out.append(dict(kind=kind, params=params, h=hs[i % len(hs)],
                        c=float(rng.uniform(0.5, 10.0)), n_rhs=4))
    return out


def surface_extent(kind: str, params) -> float:
    """Largest coordinate magnitude on the surface (centred at the origin)."""
    if kind in ("circle", "sphere"):
        return float(params[0])
    if kind == "torus":
        return float(params[0] + params[1])
    return float(max(params))


def domain_box(kind: str, params, d: int, h: float, p: int):
    """Grid box [-L, L]^d: L = 2 unless the band and its interpolation cubes
    need more room, then the next multiple of 1/2."""
    need = surface_extent(kind, params) + ruuth_merriman_gamma(d, p, h) + (p + 1) * h
    L = max(2.0, math.ceil(2.0 * need) / 2.0)
    return (-L,) * d, (L,) * d


def n_subdomains_for(n_active: int, lo: int = 32, hi: int = 512) -> int:
    """clamp(2^round(log2(N_A/2048)), lo, hi)."""
    k = int(round(math.log2(max(n_active, 1) / 2048.0)))
    return int(min(max(2 ** max(k, 0), lo), hi))


def ruuth_merriman_gamma(d: int, p: int, h: float) -> float:
    """Band radius gamma = h sqrt((d-1)((p+1)/2)^2 + (1+(p+1)/2)^2)."""
    a = (p + 1) / 2.0
    return h * math.sqrt((d - 1) * a * a + (1.0 + a) ** 2)
