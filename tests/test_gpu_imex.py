"""The library's ARK IMEX integrator (cpm.Imex, C ABI cpm_imex_*) against the oracle's
ark_step with direct stage solves.

* Gray-Scott on the torus R = 1, r = 0.4, h = 0.05 (p = 3), ARK3(2)4L[2]SA, 3
  steps of dt = 1 from the seeded noise state: every species within 1e-8
  (relative, max-norm) of the oracle; the GPU's stage solves run to 1e-12.
* The forced heat equation on the unit sphere h = 0.1 with the manufactured
  solution u = sin(t) Y (Y a degree-4 harmonic, Lap Y = -20 Y, forcing
  cos(t) Y + sin(t) 20 Y): 5 steps of dt = 0.05 within 1e-8 of the oracle, and
  close to sin(t) Y.
* A spatially uniform Gray-Scott state stays uniform and follows the explicit
  tableau on the reaction ODE (A 1 = c 1 makes every diffusion term vanish).
* IMEX Euler through cpm_imex equals the oracle's IMEX Euler step.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

from oracle import imex
from paper_2110_06322_amd import cpm, gray_scott, inputs
from tests import gpu_cases as G
from tests import oracle_cases as C

pytestmark = pytest.mark.gpu
DEV = "cuda"
MU, F, K = (2e-5, 1e-5), 0.04, 0.06


def _oracle_solver(A1, n):
    Id = sp.identity(n, format="csc")
    Lap = sp.csc_matrix(Id - A1)    # A(1) = I - Lap
    cache = {}

    def solve(s, gdm, rhs):
        if gdm not in cache:
            cache[gdm] = spla.splu(sp.csc_matrix(Id - gdm * Lap))
        return cache[gdm].solve(rhs)
    return Lap, solve


@pytest.mark.parametrize("scheme", ["ark3", "euler"])
def test_gray_scott_steps_match_oracle(scheme):
    kind, params, d, h, p = "torus", (1.0, 0.4), 3, 0.05, 3
    lb = G.lib_band(kind, params, d, h, p)
    ob, E, O, A1, P = G.oracle(kind, params, d, h, p, 1.0)
    keys, pos = G.mapping(lb, ob)
    dt, nsteps = 1.0, 3
    gs = gray_scott.GrayScott(lb, MU, F, K, dt, n_parts=8, precision="fp64", mode="fp64", rtol=1e-12,
                              scheme=scheme)
    u0, v0 = inputs.gray_scott_ic(ob.active_keys, gs.seed)
    Lap, solve = _oracle_solver(A1, ob.n_active)
    ws = [u0, v0]
    for n in range(nsteps):
        st = gs.step()
        assert all(s["converged"] for s in st)
        ws = imex.ark_step(n * dt, ws, dt, list(MU), imex.gray_scott_FE(F, K), lambda x: Lap @ x, solve, scheme)
        for name, got, want in (("u", gs.u, ws[0]), ("v", gs.v, ws[1])):
            err = float(np.abs(got.cpu().numpy() - want[pos]).max() / np.abs(want).max())
            print(f"{scheme} step {n + 1} {name}: rel err {err:.2e}, iterations {[s['iterations'] for s in st]}",
                  flush=True)
            assert err <= 1e-8


def test_heat_manufactured_sphere_matches_oracle():
    kind, params, d, h, p = "sphere", (1.0,), 3, 0.1, 3
    lb = G.lib_band(kind, params, d, h, p)
    ob, E, O, A1, P = G.oracle(kind, params, d, h, p, 1.0)
    keys, pos = G.mapping(lb, ob)
    dt, nsteps = 0.05, 5
    Y = inputs.sphere_y4(ob.cp_active, 2)
    op = cpm.Operator(lb, cpm.imex_shift("ark3", dt, 1.0))
    pc = cpm.Precond(op, kind="ras", n_parts=8)
    g1 = torch.tensor(Y[pos], dtype=torch.float64, device=DEV)
    g2 = torch.tensor(20.0 * Y[pos], dtype=torch.float64, device=DEV)
    im = cpm.Imex([op], [pc], scheme="ark3", kind="heat", dt=dt, mu=(1.0,), forcing=[g1, g2])
    u = torch.zeros(lb.n_active, dtype=torch.float64, device=DEV)
    Lap, solve = _oracle_solver(A1, ob.n_active)
    uo = [np.zeros(ob.n_active)]
    for n in range(nsteps):
        st = im.step([u], t=n * dt, nsteps=1, rtol=1e-12, max_it=5000)
        assert st[0]["converged"]
        uo = imex.ark_step(n * dt, uo, dt, [1.0], imex.heat_FE(Y, 20.0 * Y), lambda x: Lap @ x, solve, "ark3")
    got = u.cpu().numpy()
    err = float(np.abs(got - uo[0][pos]).max() / np.abs(uo[0]).max())
    exact = np.sin(nsteps * dt) * Y
    err_exact = float(np.abs(uo[0] - exact).max() / np.abs(exact).max())
    print(f"heat: rel err vs oracle {err:.2e}; oracle vs sin(t) Y {err_exact:.2e}", flush=True)
    assert err <= 1e-8
    assert err_exact <= 5e-2


def test_uniform_state_follows_explicit_tableau():
    lb = G.lib_band("torus", (1.0, 0.4), 3, 0.05, 3)
    dt = 1.0
    gs = gray_scott.GrayScott(lb, MU, F, K, dt, n_parts=8, precision="fp64", mode="fp64", rtol=1e-13,
                              scheme="ark3")
    gs.u.fill_(0.7)
    gs.v.fill_(0.2)
    ws = [np.array([0.7]), np.array([0.2])]
    for n in range(4):
        gs.step()
        ws = imex.ark_step(n * dt, ws, dt, list(MU), imex.gray_scott_FE(F, K), lambda x: np.zeros_like(x),
                           lambda s, gdm, rhs: rhs, "ark3")
    for got, want in ((gs.u, ws[0][0]), (gs.v, ws[1][0])):
        g = got.cpu().numpy()
        assert np.abs(g - want).max() <= 1e-11, (g.min(), g.max(), want)
