"""The fourth-order Laplace-Beltrami grid function on the GPU (stabilized
five-point-per-axis stencil on a band of reach 2, two-kernel apply) against the
oracle, and the degree-5 second-order operator on the same path.

* Apply parity: A4 x element-wise against the oracle's assembled
  (c + 30d/(12h^2)) I - (12h^2)^-1 (16 O1 - O2) E, at 256 eps s_i with s_i the
  row's sum of absolute terms, for cubic and quintic interpolation, 1, 2 and 4
  right-hand sides; the second-order operator with quintic interpolation
  against the oracle's A.
* Solve: A4 u = f with the (O)RAS of the cubic second-order operator as
  preconditioner, against the oracle's direct solve (1e-9, max norm).
* Convergence: the surface solution (the extension E u at the closest points)
  of (c - Lap) u = f with u = sin(theta) on the circle converges at fourth order
  with quintic interpolation, at sizes beyond the oracle's direct solves.
* A batch of two fourth-order operators equals the solo solves bit for bit; the
  transposed apply and mixed batches are refused.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from oracle import fourth, surfaces
from oracle import operator as OO
from paper_2110_06322_amd import _capi, cpm, inputs
from tests import gpu_cases as G
from tests import oracle_cases as C

pytestmark = pytest.mark.gpu
DEV = "cuda"
EPS = np.finfo(np.float64).eps


def _pair(kind, params, d, h, p):
    lb = cpm.Band(kind, params, d, h, p, reach=2)
    ob = fourth.build_band_reach(surfaces.make_cp(kind, params), d, h, p, [-2.0] * d, [2.0] * d)
    return lb, ob


CASES = [("circle", (1.0,), 2, 0.05, 3), ("circle", (1.0,), 2, 0.05, 5), ("sphere", (1.0,), 3, 0.1, 3),
         ("sphere", (1.0,), 3, 0.1, 5), ("torus", (1.0, 0.4), 3, 0.05, 5)]


@pytest.mark.parametrize("case", CASES)
def test_fourth_order_apply_parity(case):
    kind, params, d, h, p = case
    c = 1.7
    G.ensure_built()
    lb, ob = _pair(*case)
    keys, pos = G.mapping(lb, ob)
    E = OO.assemble_E(ob)
    A = fourth.assemble_A4(ob, c, E)
    O1 = fourth.assemble_O_step(ob, 1)
    O2 = fourth.assemble_O_step(ob, 2)
    w = 1.0 / (12 * h * h)
    op = cpm.Operator(lb, c, order=4)
    for nrhs in (1, 2, 4):
        xs = [G.field(ob.active_keys, 40 + q) for q in range(nrhs)]
        X = torch.tensor(np.stack([x[pos] for x in xs], axis=1).ravel(), dtype=torch.float64, device=DEV)
        Y = op.apply(X, nrhs=nrhs).cpu().numpy().reshape(-1, nrhs)
        worst = 0.0
        for q in range(nrhs):
            ax = np.abs(xs[q])
            s = (c + 30 * d * w) * ax + w * ((16 * O1 + O2) @ (abs(E) @ ax))
            worst = max(worst, float((np.abs(Y[:, q] - (A @ xs[q])[pos]) / s[pos]).max()))
        print(f"{kind} h={h} p={p} nrhs={nrhs}: N_A={lb.n_active}, max err / s_i = {worst / EPS:.2f} eps", flush=True)
        assert worst <= 256 * EPS
    # extension values of the two-kernel path's band (test hook)
    akeys, apos = G.all_mapping(lb, ob)
    x0 = torch.tensor(G.field(ob.active_keys, 40)[pos], dtype=torch.float64, device=DEV)
    v = op.extend(x0).cpu().numpy()
    xo = G.field(ob.active_keys, 40)
    assert (np.abs(v - (E @ xo)[apos]) <= 64 * EPS * (abs(E) @ np.abs(xo))[apos]).all()


def test_second_order_quintic_apply_parity():
    kind, params, d, h, p, c = "sphere", (1.0,), 3, 0.1, 5, 1.3
    G.ensure_built()
    lb = cpm.Band(kind, params, d, h, p)
    ob = C.band(kind, params, d, h, p)
    keys, pos = G.mapping(lb, ob)
    E = OO.assemble_E(ob)
    O = OO.assemble_O(ob)
    A = OO.assemble_A(ob, c, E, O)
    op = cpm.Operator(lb, c)
    xo = G.field(ob.active_keys, 7)
    y = op.apply(torch.tensor(xo[pos], dtype=torch.float64, device=DEV)).cpu().numpy()
    err = np.max(np.abs(y - (A @ xo)[pos]) / G.apply_bound(ob, E, O, c, xo)[pos])
    print(f"sphere h=0.1 p=5 order 2: max err / s_i = {err / EPS:.2f} eps", flush=True)
    assert err <= 256 * EPS


@pytest.mark.parametrize("case", [("circle", (1.0,), 2, 0.05, 5), ("sphere", (1.0,), 3, 0.1, 5)])
def test_fourth_order_solve_matches_direct(case):
    kind, params, d, h, p = case
    c = 1.0
    G.ensure_built()
    lb, ob = _pair(*case)
    keys, pos = G.mapping(lb, ob)
    inv = np.argsort(pos)
    A = fourth.assemble_A4(ob, c)
    fo = G.field(ob.active_keys, 5)
    uo = spla.spsolve(A.tocsc(), fo)
    op = cpm.Operator(lb, c, order=4)
    pc = cpm.Precond(op, kind="oras", n_parts=4 if d == 2 else 8, overlap=2.0, precision="fp64")
    f = torch.tensor(fo[pos], dtype=torch.float64, device=DEV)
    u, st = cpm.solve(op, f, pc=pc, rtol=1e-11, max_it=20000)
    assert st["converged"], st
    err = np.abs(u.cpu().numpy()[inv] - uo).max() / np.abs(uo).max()
    print(f"{kind} h={h} p={p}: {st['iterations']} iterations, |u - u_direct| / |u| = {err:.2e}", flush=True)
    assert err <= 1e-9


def test_circle_surface_solution_fourth_order():
    c, errs = 1.0, []
    G.ensure_built()
    for h in (0.05, 0.025, 0.0125):
        lb = cpm.Band("circle", (1.0,), 2, h, 5, reach=2)
        _, cp, _ = lb.export()
        s = inputs.circle_sin(cp[:lb.n_active])
        op = cpm.Operator(lb, c, order=4)
        pc = cpm.Precond(op, kind="oras", n_parts=4, overlap=2.0, precision="fp64")
        f = torch.tensor((c + 1.0) * s, dtype=torch.float64, device=DEV)
        u, st = cpm.solve(op, f, pc=pc, rtol=1e-10, max_it=20000)
        assert st["converged"], st
        v = op.extend(u).cpu().numpy()[:lb.n_active]    # u at the closest points of the active nodes
        errs.append(np.abs(v - s).max())
        print(f"circle h={h} p=5: N_A={lb.n_active}, {st['iterations']} iterations, surface error {errs[-1]:.3e}",
              flush=True)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("rates", rates, flush=True)
    assert (rates > 3.5).all(), (errs, rates)


def test_fourth_order_batch_equals_solo_and_refusals():
    G.ensure_built()
    ops, pcs, fs = [], [], []
    for kind, params, h in (("sphere", (1.0,), 0.1), ("torus", (1.0, 0.4), 0.05)):
        lb = cpm.Band(kind, params, 3, h, 5, reach=2)
        op = cpm.Operator(lb, 2.0, order=4)
        ops.append(op)
        pcs.append(cpm.Precond(op, kind="oras", n_parts=8, overlap=2.0, precision="fp64"))
        fs.append(torch.tensor(G.field(lb.active_keys, 11), dtype=torch.float64, device=DEV))
    b = cpm.Batch(ops, pcs, [1, 1])
    us, stats = b.solve(fs, rtol=1e-10, max_it=20000)
    assert all(s["converged"] for s in stats), stats
    for k in range(2):
        u1, st1 = cpm.solve(ops[k], fs[k], pc=pcs[k], rtol=1e-10, max_it=20000)
        assert torch.equal(us[k], u1), k
    ys = b.apply(fs)
    for k in range(2):
        assert torch.equal(ys[k], ops[k].apply(fs[k]))
    with pytest.raises(_capi.CpmError):
        ops[0].apply_T(fs[0])
    lb2 = cpm.Band("sphere", (1.0,), 3, 0.1, 3, reach=2)
    op_fused, op_two = cpm.Operator(lb2, 2.0), cpm.Operator(lb2, 2.0, order=4)
    with pytest.raises(_capi.CpmError):
        cpm.Batch([op_fused, op_two])
    lb3 = cpm.Band("sphere", (1.0,), 3, 0.1, 3)
    with pytest.raises(_capi.CpmError):
        cpm.Operator(lb3, 2.0, order=4)     # reach-1 band
