"""Adjoint: atomic-free A^T apply and the A^T solve behind torch.autograd.

Loss L = |u - u_t|^2 with u = A(c)^-1 f. L is exactly quadratic in f, so
central differences in f are exact for any step: the step is large
(max(1, |f|_inf)) and only the solver tolerances limit agreement: forward 1e-11,
adjoint 5e-11. The attainable relative residual, about eps |A| |u| / |f| with
|A| ~ 2d/h^2, is near 1e-11 for A and 2.5e-11 to 3e-11 for A^T at h = 0.01;
with the adjoint at 1e-10 the worst of the 16 nodes already misses the bar by
a factor 1.2, the error scaling with the adjoint tolerance.
For c, central differences with step 1e-4 c. Bar: 1e-6 relative (north-star
target) against max(|g|, 1e-3 |lambda|_inf); the dense/direct oracle
adjoint at 1e-9 on a band small enough for a direct solve.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint
from paper_2110_06322_amd import cpm, inputs
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _loss(op, f, c, ut, pc, pcT, rtol=1e-11, adjoint_rtol=5e-11):
    fv = f.clone().requires_grad_(True)
    cv = torch.tensor(c, dtype=torch.float64, requires_grad=True)
    u = cpm.CPMSolve.apply(fv, cv, op, pc, pcT, cpm.SolveOptions(rtol=rtol, max_it=50000), adjoint_rtol)
    L = ((u - ut) ** 2).sum()
    L.backward()
    return float(L), fv.grad.detach(), float(cv.grad)


def test_adjoint_matches_oracle_direct_small():
    kind, params, h = "circle", (1.0,), 0.05
    lb = G.lib_band(kind, params, 2, h, 3)
    ob, E, O, A, P = G.oracle(kind, params, 2, h, 3, 1.5)
    keys, pos = G.mapping(lb, ob)
    op = cpm.Operator(lb, 1.5)
    f = torch.tensor(G.field(keys, 1), dtype=torch.float64, device=DEV)
    ut = torch.tensor(G.field(keys, 2), dtype=torch.float64, device=DEV)
    L, gf, gc = _loss(op, f, 1.5, ut, None, None)
    Lo, uo, gfo, gco = adjoint.quadratic_loss_grads(A, G.field(ob.active_keys, 1), G.field(ob.active_keys, 2))
    assert abs(L - Lo) <= 1e-9 * Lo
    assert np.abs(gf.cpu().numpy() - gfo[pos]).max() <= 1e-9 * np.abs(gfo).max()
    assert abs(gc - gco) <= 1e-9 * abs(gco)


def test_adjoint_config4_finite_differences():
    """Torus R=1, r=0.4, h=0.01, p=3, c=1: gradient in f at 16 seeded nodes and in c vs central differences."""
    lb = G.lib_band("torus", (1.0, 0.4), 3, 0.01, 3)
    _, cp, _ = lb.export()
    cpa = cp[:lb.n_active]
    op = cpm.Operator(lb, 1.0)
    pc = cpm.Precond(op, kind="ras", n_parts=128, subsolver="ilu0")
    pcT = cpm.Precond(op, kind="ras", n_parts=128, subsolver="ilu0", transpose=True)
    f = torch.tensor(inputs.torus_modes(cpa, 1.0, seed=41), dtype=torch.float64, device=DEV)
    ut = torch.tensor(inputs.torus_modes(cpa, 1.0, seed=42), dtype=torch.float64, device=DEV)
    L, gf, gc = _loss(op, f, 1.0, ut, pc, pcT)
    print(f"N_A={lb.n_active} L={L:.6e} dL/dc={gc:.6e}", flush=True)
    lam_inf = float(gf.abs().max())
    eps = max(1.0, float(f.abs().max()))
    nodes = np.random.default_rng(4).choice(lb.n_active, 16, replace=False)
    for i in nodes:
        e = torch.zeros_like(f)
        e[int(i)] = eps
        Lp, _, _ = _loss(op, f + e, 1.0, ut, pc, pcT)
        Lm, _, _ = _loss(op, f - e, 1.0, ut, pc, pcT)
        fd = (Lp - Lm) / (2 * eps)
        g = float(gf[int(i)])
        assert abs(fd - g) <= 1e-6 * max(abs(g), 1e-3 * lam_inf), (i, fd, g)
    ec = 1e-4
    Lp, _, _ = _loss(op, f, 1.0 + ec, ut, pc, pcT)
    Lm, _, _ = _loss(op, f, 1.0 - ec, ut, pc, pcT)
    fd = (Lp - Lm) / (2 * ec)
    assert abs(fd - gc) <= 1e-6 * abs(gc), (fd, gc)
