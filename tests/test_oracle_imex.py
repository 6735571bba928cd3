"""Pins of the oracle's additive Runge-Kutta IMEX stepping (CPU only).

Independent facts used: the order conditions of Runge-Kutta methods up to
order 3 for each tableau and the coupling conditions of additive methods
(exact, in rational arithmetic); stiff decay of the L-stable implicit part on
y' = lambda y; the observed order of accuracy on the Gray-Scott reaction ODE
(a spatially uniform state, since A 1 = c 1) against a high-order reference
integration; the observed order on a linear forced system whose exact solution
is known in closed form mode by mode; the IMEX Euler tableau reproducing the
oracle's separate IMEX Euler step; and the manufactured heat solution
u = sin(t) sin(theta) on the circle.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest
import scipy.integrate as si
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import imex, reaction
from paper_2110_06322_amd import inputs
from tests import oracle_cases as C


@pytest.mark.parametrize("name", ["ark3", "euler"])
def test_order_conditions_exact(name):
    t = imex.TABLEAUX[name]
    c, AE, AI, bE, bI = t["c"], t["AE"], t["AI"], t["bE"], t["bI"]
    s = len(c)
    for A in (AE, AI):
        for i in range(s):
            # internal consistency c_i = sum_j a_ij (to the rounding of the published rationals)
            assert abs(float(sum(Fr(x) for x in A[i]) - c[i])) < 1e-24
        for j in range(s):
            if A is AE:
                assert all(AE[i][j] == 0 for i in range(j + 1))   # explicit: strictly lower
    order = t["order"]
    for b in (bE, bI):
        assert abs(float(sum(b) - 1)) < 1e-24
        if order >= 2:
            assert abs(float(sum(bi * ci for bi, ci in zip(b, c)) - Fr(1, 2))) < 1e-24
        if order >= 3:
            assert abs(float(sum(bi * ci * ci for bi, ci in zip(b, c)) - Fr(1, 3))) < 1e-24
            # b^T A c = 1/6 for each tableau and across them (the additive coupling conditions)
            for A1 in (AE, AI):
                bac = sum(b[i] * A1[i][j] * c[j] for i in range(s) for j in range(s))
                assert abs(float(bac - Fr(1, 6))) < 1e-24
    # diagonally implicit with one gamma after the explicit first stage; the implicit part
    # is stiffly accurate (its last row is b^I)
    gam = [AI[i][i] for i in range(1, s)]
    assert len(set(gam)) == 1 and AI[0][0] == 0
    assert list(AI[-1]) == list(bI)


def _scalar_step(y, dt, lam, scheme):
    return imex.ark_step(0.0, [np.array([y])], dt, [1.0], lambda t, ws: [np.zeros(1)], lambda x: lam * x,
                         lambda s, gdm, rhs: rhs / (1.0 - gdm * lam), scheme)[0][0]


def test_stiff_decay():
    for lam_dt in (-1e4, -1e8):
        assert abs(_scalar_step(1.0, 1.0, lam_dt, "ark3")) < 1e-3 * 1e4 / abs(lam_dt) + 1e-12
    assert abs(_scalar_step(1.0, 1.0, -1e8, "euler")) < 1e-7


def _uniform_gs(scheme, dt, T, F=0.04, k=0.06):
    fe = imex.gray_scott_FE(F, k)
    ws = [np.array([0.7]), np.array([0.2])]
    t = 0.0
    for _ in range(int(round(T / dt))):
        ws = imex.ark_step(t, ws, dt, [2e-5, 1e-5], fe, lambda x: np.zeros_like(x),
                           lambda s, gdm, rhs: rhs, scheme)
        t += dt
    return np.array([ws[0][0], ws[1][0]])


@pytest.mark.parametrize("scheme,order", [("ark3", 3), ("euler", 1)])
def test_order_on_uniform_gray_scott(scheme, order):
    F, k, T = 0.04, 0.06, 40.0
    ref = si.solve_ivp(lambda t, y: [-y[0] * y[1] ** 2 + F * (1 - y[0]), y[0] * y[1] ** 2 - (F + k) * y[1]],
                       (0, T), [0.7, 0.2], method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1]
    dts = (2.0, 1.0, 0.5) if order == 3 else (0.25, 0.125, 0.0625)
    e = [np.abs(_uniform_gs(scheme, dt, T) - ref).max() for dt in dts]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert (np.abs(rates - order) < 0.3).all(), (e, rates)


def _linear_system(n=12, seed=0):
    """L = -Q diag(lam) Q^T with lam in [0.2, 3]; forcing cos(t) g1 + sin(t) g2."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = -rng.uniform(0.2, 3.0, n)
    return Q, lam, rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)


def _exact_linear(Q, lam, g1, g2, u0, t):
    """u' = L u + cos(t) g1 + sin(t) g2 mode by mode: q' = l q + cos t a + sin t b has the
    particular solution P cos t + S sin t with S = l P + a, -P = l S + b."""
    a, b, q0 = Q.T @ g1, Q.T @ g2, Q.T @ u0
    P = -(lam * a + b) / (1.0 + lam ** 2)
    S = lam * P + a
    q = (q0 - P) * np.exp(lam * t) + P * np.cos(t) + S * np.sin(t)
    return Q @ q


def test_order_on_forced_linear_system():
    Q, lam, g1, g2, u0 = _linear_system()
    L = Q @ np.diag(lam) @ Q.T
    T = 2.0
    ex = _exact_linear(Q, lam, g1, g2, u0, T)
    errs = []
    for dt in (0.2, 0.1, 0.05):
        ws, t = [u0.copy()], 0.0
        for _ in range(int(round(T / dt))):
            ws = imex.ark_step(t, ws, dt, [1.0], imex.heat_FE(g1, g2), lambda x: L @ x,
                               lambda s, gdm, rhs: np.linalg.solve(np.eye(len(rhs)) - gdm * L, rhs), "ark3")
            t += dt
        errs.append(np.abs(ws[0] - ex).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (rates > 2.7).all(), (errs, rates)


def test_euler_tableau_equals_imex_euler_step():
    bd, E, Om, A1, P = C.matrices("circle", (1.0,), 2, 0.1, 2, 1.0)
    n = bd.n_active
    mu, dt, F, k = (2e-3, 1e-3), 1.0, 0.04, 0.06
    lap = lambda x: x - A1 @ x   # A(1) = I - Lap
    u0, v0 = inputs.gray_scott_ic(bd.active_keys, 3)
    Id = sp.identity(n, format="csc")
    Lap = sp.csc_matrix(Id - A1)

    def solve(s, gdm, rhs):
        return spla.spsolve(sp.csc_matrix(Id - gdm * Lap), rhs)

    got = imex.ark_step(0.0, [u0, v0], dt, list(mu), imex.gray_scott_FE(F, k), lap, solve, "euler")
    su = lambda r: spla.spsolve(sp.csc_matrix(Id / (mu[0] * dt) - Lap), r)
    sv = lambda r: spla.spsolve(sp.csc_matrix(Id / (mu[1] * dt) - Lap), r)
    ref = reaction.imex_step(su, sv, u0, v0, F, k, mu, dt)
    for a, b in zip(got, ref):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_heat_manufactured_circle():
    """u_t - Lap u = (cos t + sin t) sin(theta) has u = sin(t) sin(theta); ARK3 on the CPM
    discretization (p = 3) approaches it as h and dt shrink."""
    errs = []
    for h, dt in ((0.1, 0.1), (0.05, 0.05)):
        bd, E, Om, A1, P = C.matrices("circle", (1.0,), 2, h, 3, 1.0)
        n = bd.n_active
        s = inputs.circle_sin(bd.cp_active)
        Id = sp.identity(n, format="csc")
        Lap = sp.csc_matrix(Id - A1)
        cache = {}

        def solve(sp_, gdm, rhs):
            if gdm not in cache:
                cache[gdm] = spla.splu(sp.csc_matrix(Id - gdm * Lap))
            return cache[gdm].solve(rhs)

        ws, t = [np.zeros(n)], 0.0
        for _ in range(int(round(1.0 / dt))):
            ws = imex.ark_step(t, ws, dt, [1.0], imex.heat_FE(s, s), lambda x: Lap @ x, solve, "ark3")
            t += dt
        errs.append(np.abs(ws[0] - np.sin(1.0) * s).max())
    assert errs[1] < errs[0] / 3 and errs[1] < 2e-3, errs


def _uniform(fe, w0, scheme, dt, T, mus):
    ws = [np.array([w0[0]]), np.array([w0[1]])]
    t = 0.0
    for _ in range(int(round(T / dt))):
        ws = imex.ark_step(t, ws, dt, mus, fe, lambda x: np.zeros_like(x), lambda s, gdm, rhs: rhs, scheme)
        t += dt
    return np.array([ws[0][0], ws[1][0]])


@pytest.mark.parametrize("model", ["fitzhugh_nagumo", "schnackenberg"])
def test_order_on_uniform_fhn_and_schnackenberg(model):
    """Spatially uniform states follow the reaction ODE (Lap 1 = 0): ARK3 converges to a
    DOP853 integration of the paper's reaction terms at third order."""
    if model == "fitzhugh_nagumo":
        fe, w0, T, mus = imex.fitzhugh_nagumo_FE(), (0.6, 0.1), 20.0, (1e-4, 1e-7)
        rhs = lambda t, y: [(0.1 - y[0]) * (y[0] - 1.0) * y[0] - y[1], 0.01 * (0.5 * y[0] - y[1])]
        dts = (0.5, 0.25, 0.125)
    else:
        fe, w0, T, mus = imex.schnackenberg_FE(), (0.5, 2.0), 10.0, (1e-3, 1e-1)
        rhs = lambda t, y: [0.003 - y[0] + y[0] ** 2 * y[1] + 0.06 * y[1], 0.7 - y[0] ** 2 * y[1] - 0.06 * y[1]]
        dts = (0.2, 0.1, 0.05)
    ref = si.solve_ivp(rhs, (0, T), list(w0), method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1]
    e = [np.abs(_uniform(fe, w0, "ark3", dt, T, mus) - ref).max() for dt in dts]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    print(model, e, rates)
    assert (np.abs(rates - 3) < 0.4).all(), (e, rates)


def test_reaction_fixed_points():
    """(0, 0) is a fixed point of FitzHugh-Nagumo; (d1 + d2, d2 / ((d1 + d2)^2 + lam)) of
    Schnackenberg (the two equations' sum gives u, the second then v): one ARK3 step keeps
    them to rounding."""
    fe = imex.fitzhugh_nagumo_FE()
    out = _uniform(fe, (0.0, 0.0), "ark3", 1.0, 1.0, (1e-4, 1e-7))
    assert np.abs(out).max() == 0.0
    d1, d2, lam = 0.003, 0.7, 0.06
    us = d1 + d2
    vs = d2 / (us * us + lam)
    out = _uniform(imex.schnackenberg_FE(d1, d2, lam), (us, vs), "ark3", 0.5, 2.0, (1e-3, 1e-1))
    assert np.abs(out - [us, vs]).max() <= 1e-14 * 4
