"""Pins of the oracle's operator algebra (polynomials in the Laplace-Beltrami
operator): the assembled polynomial equals repeated application; L 1 = 0 (the
extension of a constant is constant and the stencil of a constant vanishes), so
P(L) 1 = a_0 1; manufactured solutions of the shifted biharmonic equation
(c + Lap^2) u = f from surface eigenfunctions (circle: Lap sin(theta) = -sin(theta);
sphere: Lap Y_4 = -20 Y_4) converge at second order for p = 3."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import gridfunc
from paper_2110_06322_amd import inputs
from tests import oracle_cases as C


def test_polynomial_routes_agree_and_constants():
    bd, E, Om, A, P = C.matrices("sphere", (1.0,), 3, 0.2, 3, 2.5)
    L = gridfunc.laplace_beltrami(A, 2.5)
    coef = [3.0, -1.5, 0.25]
    x = inputs.normal(4, 0, bd.active_keys)
    M = gridfunc.poly_matrix(L, coef)
    y1 = M @ x
    y2 = gridfunc.poly_apply(L, coef, x)
    assert np.abs(y1 - y2).max() <= 1e-12 * np.abs(y2).max()
    one = np.ones(bd.n_active)
    assert np.abs(L @ one).max() <= 1e-9 * (6 / 0.04)
    assert np.abs(M @ one - 3.0).max() <= 1e-9 * (6 / 0.04) ** 2


def _biharm_error(kind, h, c=1.0):
    if kind == "circle":
        bd, E, Om, A, P = C.matrices("circle", (1.0,), 2, h, 3, c)
        u = inputs.circle_sin(bd.cp_active)
        lam = 1.0
    else:
        bd, E, Om, A, P = C.matrices("sphere", (1.0,), 3, h, 3, c)
        u = inputs.sphere_y4(bd.cp_active, 2)
        lam = 20.0
    L = gridfunc.laplace_beltrami(A, c)
    M = gridfunc.poly_matrix(L, [c, 0.0, 1.0])
    x = spla.spsolve(M.tocsc(), (c + lam * lam) * u)
    return np.abs(x - u).max() / np.abs(u).max()


@pytest.mark.parametrize("kind,hs", [("circle", (0.1, 0.05, 0.025)), ("sphere", (0.2, 0.1))])
def test_shifted_biharmonic_manufactured_order(kind, hs):
    e = [_biharm_error(kind, h) for h in hs]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    print(kind, e, rates)
    assert (rates > 1.6).all(), (e, rates)
