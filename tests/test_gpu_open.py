"""Open surfaces through the C ABI: a hemisphere given by a caller's closest point
callback (cpm_band_build_user), with natural Neumann, mirrored Dirichlet and the
paper's mixed rim (Dirichlet where sin(3 phi) < -0.5, Sec. 4.1.6), against the
oracle's open band.

* Band: active / ghost sets equal the oracle's; interpolation points within
  4 ulp and signs equal (the library's hemisphere scales by R/|x| where the
  oracle's divides by |x|: 1-ulp differences in a fifth of the points).
* Operator: A x, E u and A^T x element-wise against the oracle's assembled
  matrices at the closed-surface bars (256 eps s_i, 64 eps for E), on a band
  built through the same C ABI callback from the oracle's closest point
  function, so that both sides interpolate at bitwise equal points (an ulp
  in a point moves a cubic weight by up to ~2 ulp / h, above the E bar).
* Solve: ORAS-preconditioned FP64 FGMRES to 1e-12 against the oracle's direct
  solve at 1e-10 (relative, max-norm).
* Convergence: Dirichlet hemisphere with u = z (Lap u = -2u) solved at h =
  0.05 and 0.025: second-order decrease of the error.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from oracle import open_band as OBd
from oracle import operator as OO
from paper_2110_06322_amd import cpm, inputs, surfaces
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu
DEV = "cuda"
BOX = ([-1.6] * 3, [1.6] * 3)
RIMS = {"neumann": None, "dirichlet": lambda phi: np.ones_like(phi, dtype=bool),
        "mixed": lambda phi: np.sin(3.0 * phi) < -0.5}


def _pair(h, rim):
    lb = cpm.Band.from_closest_point(surfaces.hemisphere(1.0, RIMS[rim]), 3, h, 3, *BOX)
    ob = OBd.build_open_band(OBd.hemisphere(RIMS[rim]), 3, h, 3, *BOX, inputs.ruuth_merriman_gamma(3, 3, h))
    return lb, ob


@pytest.mark.parametrize("rim", ["neumann", "dirichlet", "mixed"])
def test_open_band_operator_parity(rim):
    h, c = 0.1, 1.3
    lb, ob = _pair(h, rim)
    keys, pos = G.mapping(lb, ob)
    akeys, apos = G.all_mapping(lb, ob)
    assert lb.n_active == ob.n_active and lb.n_ghost == ob.ghost_keys.size
    ip, sg = lb.export_interp()
    assert np.array_equal(sg, ob.all_sign[apos])
    assert np.abs(ip - ob.all_ip[apos]).max() <= 4 * G.EPS * 2.0
    if rim != "neumann":
        assert (sg < 0).any()
    # the operator on interpolation points equal to the oracle's
    lb = cpm.Band.from_closest_point(OBd.hemisphere(RIMS[rim]), 3, h, 3, *BOX)
    keys, pos = G.mapping(lb, ob)
    akeys, apos = G.all_mapping(lb, ob)
    ip, sg = lb.export_interp()
    assert np.array_equal(ip, ob.all_ip[apos]) and np.array_equal(sg, ob.all_sign[apos])
    E = OBd.assemble_E_open(ob)
    O = OO.assemble_O(ob)
    A = OO.assemble_A(ob, c, E, O)
    op = cpm.Operator(lb, c)
    xo = G.field(ob.active_keys, 13)
    x = torch.tensor(xo[pos], dtype=torch.float64, device=DEV)
    y = op.apply(x).cpu().numpy()
    bound = G.apply_bound(ob, E, O, c, xo)
    err = np.max(np.abs(y - (A @ xo)[pos]) / bound[pos])
    print(f"{rim}: N_A={lb.n_active}, mirrored rows {int((sg < 0).sum())}, apply err {err / G.EPS:.2f} eps", flush=True)
    assert err <= 256 * G.EPS
    v = op.extend(x).cpu().numpy()
    vb = abs(E) @ np.abs(xo)
    ev = np.max(np.abs(v - (E @ xo)[apos]) / vb[apos])
    print(f"{rim}: extension err {ev / G.EPS:.2f} eps", flush=True)
    assert ev <= 64 * G.EPS
    yt = op.apply_T(x).cpu().numpy()
    h2 = h * h
    bt = (c + 6 / h2) * np.abs(xo) + (abs(E).T @ (O.T @ np.abs(xo))) / h2
    assert (np.abs(yt - (A.T @ xo)[pos]) <= 256 * G.EPS * bt[pos]).all()


@pytest.mark.parametrize("rim", ["neumann", "dirichlet", "mixed"])
def test_open_band_solve_matches_oracle(rim):
    h, c = 0.05, 1.0
    lb, ob = _pair(h, rim)
    keys, pos = G.mapping(lb, ob)
    E = OBd.assemble_E_open(ob)
    A = OO.assemble_A(ob, c, E, OO.assemble_O(ob))
    fo = (c + 6.0) * (3.0 * ob.cp_active[:, 2] ** 2 - 1.0)
    xo = spla.spsolve(A.tocsc(), fo)
    op = cpm.Operator(lb, c)
    pc = cpm.Precond(op, kind="oras", n_parts=8, overlap=2.0)
    u, st = cpm.solve(op, torch.tensor(fo[pos], dtype=torch.float64, device=DEV), pc=pc, rtol=1e-12, max_it=20000)
    assert st["converged"], st
    err = float(np.abs(u.cpu().numpy() - xo[pos]).max() / np.abs(xo).max())
    print(f"{rim}: {st['iterations']} iterations, error vs oracle {err:.2e}", flush=True)
    assert err <= 1e-10


def test_dirichlet_hemisphere_converges_second_order():
    errs = []
    for h in (0.05, 0.025):
        lb = cpm.Band.from_closest_point(surfaces.hemisphere(1.0, RIMS["dirichlet"]), 3, h, 3, *BOX)
        _, cp, _ = lb.export()
        ip, sg = lb.export_interp()
        cpa = cp[:lb.n_active]
        op = cpm.Operator(lb, 1.0)
        pc = cpm.Precond(op, kind="ras", n_parts=16, overlap=2.0)
        f = torch.tensor(3.0 * cpa[:, 2], dtype=torch.float64, device=DEV)
        u, st = cpm.solve(op, f, pc=pc, rtol=1e-12, max_it=20000)
        assert st["converged"]
        keep = sg[:lb.n_active] > 0
        errs.append(float(np.abs(u.cpu().numpy() - cpa[:, 2])[keep].max()))
    rate = np.log2(errs[0] / errs[1])
    print("errors", errs, "order", rate, flush=True)
    assert rate > 1.5 and errs[1] < 2e-3
