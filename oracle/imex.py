"""Additive Runge-Kutta IMEX time stepping for surface reaction-diffusion systems
(paper Sec. 1, eq. rdsys; Sec. 4.1.3 heat equation eq. heat / eq. htForce,
Sec. 4.1.4 FitzHugh-Nagumo eq. fitznag, Sec. 4.1.5 Gray-Scott eq. grayscott and
Sec. 4.1.6 Schnackenberg eq. schnack, whose default PETSc integrator is the
third-order additive Runge-Kutta IMEX scheme).

For w_t = F_E(t, w) + mu Lap_S w, with the diffusion implicit and the rest
explicit, an s-stage ARK method with explicit tableau (A^E, b, c) and
singly-diagonally implicit tableau (A^I, b, c) computes
  W_1 = w^n                                             (a^I_11 = 0)
  (I - dt a^I_ii mu Lap) W_i = w^n + dt sum_{j<i} (a^E_ij K^E_j + a^I_ij K^I_j)
  K^E_j = F_E(t_n + c_j dt, W_j),  K^I_j = mu Lap W_j
  w^{n+1} = w^n + dt sum_j (b^E_j K^E_j + b^I_j K^I_j)
(b^E = b^I for the Kennedy-Carpenter scheme; IMEX Euler has b^E != b^I).
With the CPM operator A(c) = c I - Lap_S^h (eq. lapBel), each stage solve is
A(c_s) W_i = rhs / (dt gamma mu) with c_s = 1/(dt gamma mu), gamma = a^I_ii.

Tableaux (exact rationals from the publications):
  ark3: ARK3(2)4L[2]SA, Kennedy & Carpenter, "Additive Runge-Kutta schemes for
        convection-diffusion-reaction equations", Appl. Numer. Math. 44 (2003),
        the four-stage third-order scheme with an L-stable, stiffly accurate
        ESDIRK part;
  euler: IMEX Euler (forward Euler for F_E, backward Euler for the diffusion)
        as a two-stage ARK tableau.
"""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np

_G = Fr(1767732205903, 4055673282236)

TABLEAUX = {
    "ark3": {
        "c": [Fr(0), Fr(1767732205903, 2027836641118), Fr(3, 5), Fr(1)],
        "AI": [[Fr(0), 0, 0, 0],
               [_G, _G, 0, 0],
               [Fr(2746238789719, 10658868560708), Fr(-640167445237, 6845629431997), _G, 0],
               [Fr(1471266399579, 7840856788654), Fr(-4482444167858, 7529755066697),
                Fr(11266239266428, 11593286722821), _G]],
        "AE": [[Fr(0), 0, 0, 0],
               [Fr(1767732205903, 2027836641118), 0, 0, 0],
               [Fr(5535828885825, 10492691773637), Fr(788022342437, 10882634858940), 0, 0],
               [Fr(6485989280629, 16251701735622), Fr(-4246266847089, 9704473918619),
                Fr(10755448449292, 10357097424841), 0]],
        "bE": [Fr(1471266399579, 7840856788654), Fr(-4482444167858, 7529755066697),
               Fr(11266239266428, 11593286722821), _G],
        "bI": [Fr(1471266399579, 7840856788654), Fr(-4482444167858, 7529755066697),
               Fr(11266239266428, 11593286722821), _G],
        "order": 3,
    },
    "euler": {
        "c": [Fr(0), Fr(1)],
        "AI": [[Fr(0), 0], [Fr(0), Fr(1)]],
        "AE": [[Fr(0), 0], [Fr(1), 0]],
        "bE": [Fr(1), Fr(0)],
        "bI": [Fr(0), Fr(1)],
        "order": 1,
    },
}


def tableau(name: str):
    """(c, AE, AI, bE, bI) as float64 arrays."""
    t = TABLEAUX[name]
    vec = lambda v: np.array([float(x) for x in v])
    return (vec(t["c"]), np.array([vec(r) for r in t["AE"]]), np.array([vec(r) for r in t["AI"]]),
            vec(t["bE"]), vec(t["bI"]))


def ark_step(t, ws, dt, mus, FE, lap, solve, scheme="ark3"):
    """One ARK IMEX step of a system of species.

    ws: list of arrays (state of each species); mus: diffusion coefficients;
    FE(t, Ws) -> list of arrays (explicit terms, all species); lap(x) = Lap_S^h x;
    solve(s, gamma_dt_mu, rhs) solves (I - gamma_dt_mu Lap_S^h) W = rhs for species s.
    Returns the new list of arrays.
    """
    c, AE, AI, bE, bI = tableau(scheme)
    ns = len(ws)
    st = len(c)
    W = [list(ws)]
    KE = [FE(t, ws)]
    KI = [[mus[s] * lap(ws[s]) for s in range(ns)]]
    for i in range(1, st):
        Wi = []
        for s in range(ns):
            rhs = ws[s].copy()
            for j in range(i):
                rhs = rhs + dt * (AE[i, j] * KE[j][s] + AI[i, j] * KI[j][s])
            Wi.append(solve(s, dt * AI[i, i] * mus[s], rhs))
        W.append(Wi)
        KE.append(FE(t + c[i] * dt, Wi))
        KI.append([mus[s] * lap(Wi[s]) for s in range(ns)])
    out = []
    for s in range(ns):
        acc = ws[s].copy()
        for j in range(st):
            acc = acc + dt * (bE[j] * KE[j][s] + bI[j] * KI[j][s])
        out.append(acc)
    return out


def gray_scott_FE(F, k):
    """Explicit terms of the Gray-Scott system (eq. grayscott): the reaction."""
    def fe(t, ws):
        u, v = ws
        uv2 = u * v * v
        return [-uv2 + F * (1.0 - u), uv2 - (F + k) * v]
    return fe


def heat_FE(g_cos, g_sin):
    """Explicit term of the forced heat equation u_t - Lap_S u = f (eq. heat) with
    f(x, t) = cos(t) g_cos(x) + sin(t) g_sin(x) (eq. htForce has this form)."""
    def fe(t, ws):
        return [np.cos(t) * g_cos + np.sin(t) * g_sin]
    return fe


def fitzhugh_nagumo_FE(a=0.1, eps=0.01, beta=0.5):
    """Explicit terms of the FitzHugh-Nagumo system (Sec. 4.1.4, eq. fitznag):
    u_t - D_u Lap u = (a - u)(u - 1) u - v,  v_t - D_v Lap v = eps (beta u - v)
    (the paper's values a = 0.1, eps = 0.01, beta = 0.5)."""
    def fe(t, ws):
        u, v = ws
        return [(a - u) * (u - 1.0) * u - v, eps * (beta * u - v)]
    return fe


def schnackenberg_FE(delta1=0.003, delta2=0.7, lam=0.06):
    """Explicit terms of the Schnackenberg system (Sec. 4.1.6, eq. schnack):
    u_t - D_u Lap u = delta1 - u + u^2 v + lam v,  v_t - D_v Lap v = delta2 - u^2 v - lam v."""
    def fe(t, ws):
        u, v = ws
        u2v = u * u * v
        return [delta1 - u + u2v + lam * v, delta2 - u2v - lam * v]
    return fe
