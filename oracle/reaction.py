"""Semi-implicit (IMEX Euler) step of the Gray-Scott system on a surface
(paper Sec. 1, eq. rdsys; Sec. 4.1.5, eq. grayscott: reaction explicit, diffusion implicit).

  u_t - mu_u Lap_S u = -u v^2 + F (1 - u)
  v_t - mu_v Lap_S v =  u v^2 - (F + k) v
IMEX Euler with the shifted CPM operator A_w = c_w I - Delta_S^h, c_w = 1/(mu_w dt):
  (1/dt - mu_w Delta_S^h) w^{n+1} = w^n/dt + R_w(u^n, v^n)
  <=> A_w w^{n+1} = (w^n/dt + R_w(u^n, v^n)) / mu_w.
"""
from __future__ import annotations

import numpy as np


def gray_scott_reaction(u, v, F, k):
    uv2 = u * v * v
    return -uv2 + F * (1.0 - u), uv2 - (F + k) * v


def imex_rhs(u, v, F, k, mu, dt):
    Ru, Rv = gray_scott_reaction(u, v, F, k)
    return (u / dt + Ru) / mu[0], (v / dt + Rv) / mu[1]


def imex_step(solve_u, solve_v, u, v, F, k, mu, dt):
    """One step; solve_w(rhs) must solve (1/(mu_w dt) - Delta_S^h) w = rhs."""
    fu, fv = imex_rhs(u, v, F, k, mu, dt)
    return solve_u(fu), solve_v(fv)
