"""Pins of the oracle's closest point functions and band (CPU only).

Fixed independently of the oracle by: the defining minimisation property of
cp (on the surface, x - cp along the normal, nearer than sampled surface
points), special cases (ellipsoid with equal axes = sphere), tube-volume
closed forms for the band size, and the inclusion of every band node's
interpolation cube and neighbours in the band (paper Sec. 2.1).
"""
import math

import numpy as np
import pytest

from oracle import band as B
from oracle import surfaces
from paper_2110_06322_amd import inputs
from tests import oracle_cases as C

rng = np.random.default_rng(0)


def test_sphere_cp_minimises_distance():
    x = rng.uniform(-2, 2, size=(200, 3))
    cp = surfaces.cp_sphere(x, (0.0, 0.0, 0.0), 1.0)
    assert np.allclose(np.linalg.norm(cp, axis=1), 1.0, atol=1e-15)
    th = rng.uniform(0, math.pi, 4000)
    ph = rng.uniform(0, 2 * math.pi, 4000)
    S = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    dmin = np.linalg.norm(x[:, None, :] - S[None], axis=2).min(axis=1)
    assert (np.linalg.norm(x - cp, axis=1) <= dmin + 1e-14).all()


def test_torus_cp_on_surface_and_normal():
    R, r = 1.0, 0.4
    x = rng.uniform(-1.6, 1.6, size=(300, 3))
    x = x[np.hypot(x[:, 0], x[:, 1]) > 0.7]
    cp = surfaces.cp_torus(x, R, r)
    rho = np.hypot(cp[:, 0], cp[:, 1])
    assert np.allclose((rho - R) ** 2 + cp[:, 2] ** 2, r * r, atol=1e-14)
    # gradient of the implicit function (rho - R)^2 + z^2 - r^2 at cp
    g = np.stack([2 * (rho - R) * cp[:, 0] / rho, 2 * (rho - R) * cp[:, 1] / rho, 2 * cp[:, 2]], 1)
    assert np.abs(np.cross(x - cp, g)).max() < 1e-12
    u = rng.uniform(0, 2 * math.pi, (2, 20000))
    S = np.stack([(R + r * np.cos(u[1])) * np.cos(u[0]), (R + r * np.cos(u[1])) * np.sin(u[0]),
                  r * np.sin(u[1])], 1)
    dmin = np.linalg.norm(x[:, None, :] - S[None], axis=2).min(axis=1)
    assert (np.linalg.norm(x - cp, axis=1) <= dmin + 1e-12).all()


def test_ellipsoid_cp_property_and_sphere_case():
    axes = (1.3, 0.8, 0.65)
    a = np.array(axes)
    # points near the surface (the band), inside and outside
    d = rng.standard_normal((400, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    x = d * a[None, :] * rng.uniform(0.85, 1.15, (400, 1))
    cp = surfaces.cp_ellipsoid(x, axes)
    assert np.allclose(((cp / a) ** 2).sum(1), 1.0, atol=1e-14)
    g = 2 * cp / (a * a)
    assert np.abs(np.cross(x - cp, g)).max() < 1e-12
    # brute force over a dense parametrisation
    u = rng.uniform(0, 1, (2, 60000))
    th = np.arccos(1 - 2 * u[0])
    ph = 2 * math.pi * u[1]
    S = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1) * a
    dmin = np.linalg.norm(x[:50, None, :] - S[None], axis=2).min(axis=1)
    assert (np.linalg.norm(x[:50] - cp[:50], axis=1) <= dmin + 1e-12).all()
    # equal axes: the sphere's radial projection
    cps = surfaces.cp_ellipsoid(x, (1.0, 1.0, 1.0))
    assert np.abs(cps - surfaces.cp_sphere(x, (0, 0, 0), 1.0)).max() < 1e-14


def test_ellipsoid_cp_near_and_on_the_medial_set():
    """Interior points beside the plane of the smallest axis have their closest
    point off that plane (brute force decides); points on the plane inside the
    medial set have two mirror closest points and get NaN; points on the plane
    outside it keep a unique closest point in the plane."""
    axes = (1.2410195721651176, 1.0657296288514941, 0.6753029137923193)
    a = np.array(axes)
    near = np.array([[0.1, -0.3, 1e-6], [0.0, -0.4, -1e-4], [0.3, 0.2, 1e-3], [-0.2, 0.0, 2e-3]])
    onplane_medial = np.array([[0.0, -0.4, 0.0], [0.1, 0.0, 0.0], [0.0, 0.0, 0.0], [0.3, 0.2, 0.0]])
    onplane_unique = np.array([[0.0, 0.9, 0.0], [1.1, 0.0, 0.0], [1.5, 0.5, 0.0]])
    u = rng.uniform(0, 1, (2, 200000))
    th = np.arccos(1 - 2 * u[0])
    ph = 2 * math.pi * u[1]
    S = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1) * a
    for x in (near, onplane_unique):
        cp = surfaces.cp_ellipsoid(x, axes)
        assert np.allclose(((cp / a) ** 2).sum(1), 1.0, atol=1e-13)
        dmin = np.linalg.norm(x[:, None, :] - S[None], axis=2).min(axis=1)
        dcp = np.linalg.norm(x - cp, axis=1)
        assert (dcp <= dmin + 1e-12).all() and (dcp >= dmin - 2e-3).all()
    assert np.isnan(surfaces.cp_ellipsoid(onplane_medial, axes)).all()


@pytest.mark.parametrize("kind,params,d,h,p,area", [
    ("circle", (1.0,), 2, 0.05, 2, None),
    ("circle", (1.0,), 2, 0.025, 3, None),
    ("sphere", (1.0,), 3, 0.04, 3, None),
    ("torus", (1.0, 0.4), 3, 0.05, 3, None),
])
def test_band_size_matches_tube_volume(kind, params, d, h, p, area):
    bd = C.band(kind, params, d, h, p)
    g = bd.gamma
    if kind == "circle":
        vol = math.pi * ((1 + g) ** 2 - (1 - g) ** 2) / h ** 2
    elif kind == "sphere":
        vol = 4.0 / 3.0 * math.pi * ((1 + g) ** 3 - (1 - g) ** 3) / h ** 3
    else:
        R, r = params
        vol = 2 * math.pi * R * math.pi * ((r + g) ** 2 - (r - g) ** 2) / h ** 3
    assert abs(bd.n_band - vol) / vol < 0.01


def test_band_circle_h005_sizes():
    bd = C.band("circle", (1.0,), 2, 0.05, 2)
    assert (bd.n_band, bd.n_active, bd.n_ghost) == (732, 464, 228)


@pytest.mark.parametrize("kind,params,d,h,p", [
    ("circle", (1.0,), 2, 0.05, 2),
    ("sphere", (1.0,), 3, 0.1, 3),
    ("torus", (1.0, 0.4), 3, 0.05, 3),
    ("ellipsoid", (1.3, 0.8, 0.65), 3, 0.05, 3),
])
def test_band_closure_and_inclusion(kind, params, d, h, p):
    """Every node of Sigma_A u Sigma_G lies in B_gamma, its cube lies in Sigma_A,
    and the neighbours of Sigma_A lie in Sigma_A u Sigma_G; no closure step was needed."""
    bd = C.band(kind, params, d, h, p)
    assert bd.closure_iterations == 0
    x = B.coords(bd.all_ijk, bd.lo, h)
    dist = np.linalg.norm(x - bd.all_cp, axis=1)
    assert (dist <= bd.gamma * (1 + 1e-10)).all()
    base = B.stencil_base(bd.all_cp, bd.lo, h, p)
    offs = B.cube_offsets(d, p)
    cube = B.keys_of((base[:, None, :] + offs[None]).reshape(-1, d), bd.shape)
    assert np.isin(cube, bd.active_keys).all()
    allk = bd.all_keys
    for k in range(d):
        for s in (-1, 1):
            nb = bd.active_ijk.copy()
            nb[:, k] += s
            assert np.isin(B.keys_of(nb, bd.shape), allk).all()
    assert np.intersect1d(bd.active_keys, bd.ghost_keys).size == 0


def test_grid_node_closest_point_is_exact():
    """On the unit circle at h = 0.05 the node (1.1, 0) projects onto (1, 0) to within an ulp."""
    bd = C.band("circle", (1.0,), 2, 0.05, 2)
    ijk, cp = bd.all_ijk, bd.all_cp
    i = np.nonzero((ijk[:, 0] == 62) & (ijk[:, 1] == 40))[0]
    assert i.size == 1
    assert cp[i[0], 1] == 0.0 and abs(cp[i[0], 0] - 1.0) <= 2.3e-16


def test_gamma_formula():
    assert abs(inputs.ruuth_merriman_gamma(2, 2, 0.05) - 0.05 * math.sqrt(1 * 1.5 ** 2 + 2.5 ** 2)) < 1e-16
    assert abs(inputs.ruuth_merriman_gamma(3, 3, 0.02) / 0.02 - math.sqrt(17)) < 1e-12
