"""Semi-implicit Gray-Scott on a torus: the library kernels against the oracle.

Pins: a spatially uniform state stays uniform and follows the explicit-Euler
reaction ODE exactly (A 1 = c 1), to the solver tolerance; for seeded noise,
the first steps agree with the oracle's IMEX step (direct solves) to 1e-8
relative (solver rtol 1e-11, pattern formation has not amplified rounding yet);
checkpoint and resume reproduce the trajectory bit for bit.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

from oracle import reaction
from paper_2110_06322_amd import cpm, gray_scott, inputs
from tests import gpu_cases as G
from tests import oracle_cases as C

pytestmark = pytest.mark.gpu
MU, F, K, DT = (2e-5, 1e-5), 0.04, 0.06, 1.0


def _sim(h=0.05, n_parts=8, rtol=1e-11, mode="fp64", precision="fp64"):
    G.ensure_built()
    b = G.lib_band("torus", (1.0, 0.4), 3, h, 3)
    return b, gray_scott.GrayScott(b, MU, F, K, DT, n_parts=n_parts, precision=precision, mode=mode, rtol=rtol)


def test_uniform_state_follows_reaction_ode():
    b, gs = _sim()
    gs.u.fill_(0.7)
    gs.v.fill_(0.2)
    uu, vv = 0.7, 0.2
    for _ in range(4):
        gs.step()
        Ru, Rv = reaction.gray_scott_reaction(uu, vv, F, K)
        uu, vv = uu + DT * Ru, vv + DT * Rv
    assert float((gs.u - uu).abs().max()) <= 1e-9
    assert float((gs.v - vv).abs().max()) <= 1e-9


def test_first_steps_match_oracle_and_checkpoint(tmp_path):
    b, gs = _sim()
    ob, E, O, A0, P = C.matrices("torus", (1.0, 0.4), 3, 0.05, 3, 1.0)
    keys, pos = G.mapping(b, ob)
    n = ob.n_active
    Ip = sp.identity(n, format="csr")
    su = spla.factorized((A0 - Ip + (1.0 / (MU[0] * DT)) * Ip).tocsc())
    sv = spla.factorized((A0 - Ip + (1.0 / (MU[1] * DT)) * Ip).tocsc())
    u0, v0 = inputs.gray_scott_ic(ob.active_keys, gs.seed)
    uo, vo = u0, v0
    for step in range(3):
        gs.step()
        uo, vo = reaction.imex_step(su, sv, uo, vo, F, K, MU, DT)
        du = np.abs(gs.u.cpu().numpy() - uo[pos]).max() / np.abs(uo).max()
        dv = np.abs(gs.v.cpu().numpy() - vo[pos]).max() / np.abs(vo).max()
        print(f"step {step}: u {du:.2e} v {dv:.2e} iterations {[s['iterations'] for s in gs.last_stats]}")
        assert du <= 1e-8 and dv <= 1e-8
    ck = tmp_path / "gs.npz"
    gs.checkpoint(ck)
    gs.step()
    u_ref, v_ref = gs.u.clone(), gs.v.clone()
    _, gs2 = _sim()
    gs2.resume(ck)
    assert gs2.step_count == 3
    gs2.step()
    assert torch.equal(gs2.u, u_ref) and torch.equal(gs2.v, v_ref)


def test_mixed_precision_steps_stay_close_to_fp64():
    b, g64 = _sim(rtol=1e-10)
    _, g32 = _sim(rtol=1e-10, mode="mixed", precision="fp32")
    for _ in range(3):
        g64.step()
        g32.step()
    d = float((g64.u - g32.u).abs().max())
    print(f"mixed vs fp64 after 3 steps: {d:.2e}")
    assert d <= 1e-8
