"""Pins of the oracle's fourth-order Laplace-Beltrami grid function (CPU only).

Independent facts used: the textbook fourth-order periodic second difference,
whose symbol at frequency theta is -(30 - 32 cos(theta) + 2 cos(2 theta))/(12 h^2),
solves the system on a grid-aligned periodic line in closed form (FFT); A4 1 = c 1
(the stencil weights sum to zero and E reproduces constants); the ghost set holds
every node within two steps of Sigma_A and the closure property; the observed
order of accuracy on the circle eigenfunction sin(theta) (Lap = -1) of the surface
solution, i.e. the discrete solution interpolated at the closest points (E u):
fourth order with quintic interpolation, second order with cubic (the
interpolation error O(h^{p+1}) divided by h^2 dominates). The node values off the
surface carry an O(h^3) part (the stencil sees the Laplacian of the parallel
curve through the node, O(distance) from the surface one, damped by the O(h^-2)
diagonal), which the interpolation to the surface does not see.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import band as B
from oracle import fourth, surfaces
from oracle import operator as OO
from paper_2110_06322_amd import inputs


@pytest.mark.parametrize("p", [3, 5])
def test_periodic_line_reduces_to_textbook_fourth_order_difference(p):
    h, n, y0, c = 0.0625, 64, 0.5, 3.0
    lo, hi = [0.0, 0.0], [(n - 1) * h, 1.0]
    bd = fourth.build_band_reach(surfaces.make_cp("line", (y0,)), 2, h, p, lo, hi, reach=2,
                                 periodic=(True, False))
    A = fourth.assemble_A4(bd, c)
    X = bd.active_ijk[:, 0] * h
    L = n * h
    F = np.cos(2 * math.pi * 3 * X / L) + 0.3 * np.sin(2 * math.pi * 7 * X / L)
    u = spla.spsolve(A.tocsc(), F)
    xs = np.arange(n) * h
    Fl = np.cos(2 * math.pi * 3 * xs / L) + 0.3 * np.sin(2 * math.pi * 7 * xs / L)
    th = 2 * math.pi * np.arange(n) / n
    sym = c + (30.0 - 32.0 * np.cos(th) + 2.0 * np.cos(2.0 * th)) / (12.0 * h * h)
    U = np.fft.ifft(np.fft.fft(Fl) / sym).real
    assert np.abs(u - U[bd.active_ijk[:, 0]]).max() < 1e-12


def test_constants_band_sets_and_closure():
    h, p, c = 0.2, 3, 1.7
    cpf = surfaces.make_cp("sphere", (1.0,))
    bd = fourth.build_band_reach(cpf, 3, h, p, [-2.0] * 3, [2.0] * 3)
    A = fourth.assemble_A4(bd, c)
    one = np.ones(bd.n_active)
    assert np.abs(A @ one - c).max() <= 1e-9 * (30 * 3 / (12 * h * h))
    # every node within two steps along an axis of Sigma_A is active or ghost, and only those
    act = set(bd.active_keys.tolist())
    need = set()
    for k in range(3):
        for s in (-2, -1, 1, 2):
            q = bd.active_ijk.copy()
            q[:, k] += s
            need.update(B.keys_of(q, bd.shape).tolist())
    assert set(bd.ghost_keys.tolist()) == need - act
    # closure: every cube of every band node lies in Sigma_A
    cubes = B._cubes(bd.all_cp, bd.lo, h, p, bd.shape, ())
    assert set(np.unique(cubes).tolist()) <= act
    # the second-order band's sets are subsets (same radius): the ghost layer only grew
    b1 = B.build_band(cpf, 3, h, p, [-2.0] * 3, [2.0] * 3, fourth.gamma_reach(3, p, h, 2))
    assert set(b1.active_keys.tolist()) <= act
    assert set(b1.ghost_keys.tolist()) <= set(bd.ghost_keys.tolist())


def _circle_error(h, p, c=1.0):
    bd = fourth.build_band_reach(surfaces.make_cp("circle", (1.0,)), 2, h, p, [-2.0, -2.0], [2.0, 2.0])
    A = fourth.assemble_A4(bd, c)
    s = inputs.circle_sin(bd.cp_active)
    u = spla.spsolve(A.tocsc(), (c + 1.0) * s)
    v = (OO.assemble_E(bd) @ u)[:bd.n_active]   # u at the closest points of the active nodes
    return np.abs(v - s).max()


def test_circle_fourth_order_with_quintic_interpolation():
    e = [_circle_error(h, 5) for h in (0.1, 0.05, 0.025)]
    rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    print("p=5", e, rates)
    assert all(r > 3.5 for r in rates), (e, rates)


def test_circle_second_order_with_cubic_interpolation():
    e = [_circle_error(h, 3) for h in (0.1, 0.05, 0.025)]
    rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    print("p=3", e, rates)
    assert all(1.7 < r < 2.6 for r in rates), (e, rates)
