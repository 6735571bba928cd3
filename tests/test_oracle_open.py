"""Pins of the oracle's open-surface band (hemisphere with Neumann / Dirichlet rims).

Independent facts used: the closest point minimises the distance over a dense
sampling of the hemisphere; mirrored nodes interpolate at a point of the cap
with weight sign -1, so every extension row sums to its sign; the Laplace-
Beltrami eigenfunctions of the unit sphere restricted to the upper hemisphere:
3 z^2 - 1 (eigenvalue 6) has zero normal derivative on the rim (Neumann) and
z (eigenvalue 2) vanishes on it (Dirichlet), so (c - Lap) u = (c + l(l+1)) u
is solved by them and the discrete solutions converge to them as h shrinks.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import open_band as OB
from oracle import operator as OO
from paper_2110_06322_amd import inputs


def test_hemisphere_closest_points_minimise_distance():
    rng = np.random.default_rng(1)
    x = rng.uniform(-1.6, 1.6, (400, 3))
    x = x[np.linalg.norm(x, axis=1) > 0.3]
    cp, flag = OB.hemisphere()(x)
    th = rng.uniform(0, np.pi / 2, 200000)
    ph = rng.uniform(-np.pi, np.pi, 200000)
    S = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    rim = np.stack([np.cos(ph), np.sin(ph), np.zeros_like(ph)], axis=1)
    S = np.concatenate([S, rim])
    for xi, ci in zip(x, cp):
        assert abs(np.linalg.norm(ci) - 1.0) < 1e-14 and ci[2] >= 0.0
        dmin = np.sqrt(((S - xi) ** 2).sum(axis=1)).min()
        assert np.linalg.norm(xi - ci) <= dmin + 1e-12
    assert (flag == 0).all()


def _band(h, dirichlet):
    f = OB.hemisphere(dirichlet)
    return OB.build_open_band(f, 3, h, 3, [-1.6] * 3, [1.6] * 3, inputs.ruuth_merriman_gamma(3, 3, h))


def test_mirrored_rows_interpolate_on_the_cap_and_sum_to_their_sign():
    bd = _band(0.1, lambda phi: np.ones_like(phi, dtype=bool))
    s = bd.all_sign
    assert (s == -1).any() and (s == 1).any()
    ip = bd.all_ip
    m = s < 0
    assert np.abs(np.linalg.norm(ip[m], axis=1) - 1.0).max() < 1e-14
    assert (ip[m][:, 2] >= 0).all()   # on the cap (the rim itself for nodes on the plane z = 0)
    # mirrored exactly the nodes whose closest point is on the rim
    cp = np.concatenate([bd.cp_active, bd.cp_ghost])
    assert np.array_equal(m, cp[:, 2] == 0.0)
    E = OB.assemble_E_open(bd)
    assert np.abs(np.asarray(E.sum(axis=1)).ravel() - s).max() < 1e-14


def _solve(h, bc, c=1.0):
    if bc == "neumann":
        bd = _band(h, None)
        u = lambda q: 3.0 * q[:, 2] ** 2 - 1.0
        lam = 6.0
    else:
        bd = _band(h, lambda phi: np.ones_like(phi, dtype=bool))
        u = lambda q: q[:, 2]
        lam = 2.0
    E = OB.assemble_E_open(bd)
    O = OO.assemble_O(bd)
    A = OO.assemble_A(bd, c, E, O)
    f = (c + lam) * u(bd.cp_active)
    x = spla.spsolve(A.tocsc(), f)
    keep = bd.sign_active > 0
    return np.abs(x - u(bd.cp_active))[keep].max()


@pytest.mark.parametrize("bc,min_order,bar", [("neumann", 0.8, 0.25), ("dirichlet", 1.5, 0.02)])
def test_hemisphere_manufactured_convergence(bc, min_order, bar):
    """The natural (Neumann) treatment is first-order accurate and its boundary error reaches
    the whole surface; the mirrored (Dirichlet) one is second order."""
    e = [_solve(h, bc) for h in (0.2, 0.1, 0.05)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    print(bc, e, rates)
    assert e[-1] < bar and (rates > min_order).all(), (e, rates)
