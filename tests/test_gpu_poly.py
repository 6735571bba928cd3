"""Operator algebra on the GPU: polynomials in the Laplace-Beltrami operator
L = c I - A(c) (sums and compositions of the identity and L; the shifted
biharmonic c0 + L^2), applied by cpm_poly_apply and solved by FGMRES with the
(O)RAS preconditioner of A(sqrt(c0)) applied twice.

* Parity of P(L) x with the oracle's repeated products, for the coefficient
  lists [a0], [a0, a1], ... of every degree up to 4 (so that each term is
  larger than the tolerance of the list it is added in), 1, 2 and 4
  right-hand sides, on a circle, a sphere and a torus. Bar per entry:
  256 eps sum_k |a_k| (|L|^k |x|), a forward-error bound of the products;
  degree 0 is bit-exact.
* The shifted biharmonic solve (c0 = 1) on the sphere h = 0.1 against the
  oracle's sparse direct solve of the assembled c0 I + L L: true residual by
  the oracle's matrix within the solve tolerance, solution within 1e-7.
* Second-order convergence of the shifted biharmonic on manufactured surface
  eigenfunctions (circle h = 0.1 / 0.05 / 0.025, sphere h = 0.1 / 0.05; the
  oracle's direct solves give the same errors where they fit, e.g. 0.71 on the
  sphere at h = 0.1: Y_4 has biharmonic eigenvalue 400). These and the batch
  use the two-level (coarse-first) ORAS of A(sqrt(c0)) twice and GMRES(60): with
  one level, the squared preconditioner leaves GMRES(30) stagnating from
  h = 0.05 on (the one-level iteration growth with the subdomain count is
  squared as well).
  Tolerances respect the attainable residual: c0 + L^2 has norm ~ (4d/h^2)^2,
  so FP64 rounding of its application alone leaves a relative residual of
  about eps (4d/h^2)^2 |u| / |f|; the solve tolerance stays above it, and the
  error it allows (|e| <= |r| / c0) stays far below the discretization error.
* A batch of two surfaces solving c0 + L^2 together equals the solo solves bit
  for bit.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

from oracle import gridfunc
from paper_2110_06322_amd import _capi, cpm, inputs
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu
DEV = "cuda"
EPS = np.finfo(np.float64).eps
COEF = [3.0, -1.5, 0.25, -0.01, 2e-4]


@pytest.mark.parametrize("case", [("circle", (1.0,), 2, 0.03, 3), ("sphere", (1.0,), 3, 0.1, 3),
                                  ("torus", (1.0, 0.4), 3, 0.05, 3)])
@pytest.mark.parametrize("nrhs", [1, 2, 4])
def test_poly_apply_parity(case, nrhs):
    kind, params, d, h, p = case
    c = 2.5
    lb = G.lib_band(kind, params, d, h, p)
    ob, E, O, A, P = G.oracle(kind, params, d, h, p, c)
    keys, pos = G.mapping(lb, ob)
    op = cpm.Operator(lb, c)
    L = gridfunc.laplace_beltrami(A, c)
    absL = abs(L)
    xs = [G.field(ob.active_keys, 80 + q) for q in range(nrhs)]
    X = torch.tensor(np.stack([x[pos] for x in xs], axis=1).ravel(), dtype=torch.float64, device=DEV)
    for deg in range(len(COEF)):
        coef = COEF[:deg + 1]
        Y = op.poly_apply(coef, X, nrhs=nrhs).cpu().numpy().reshape(-1, nrhs)
        worst = 0.0
        for q in range(nrhs):
            yo = gridfunc.poly_apply(L, coef, xs[q])[pos]
            if deg == 0:
                assert np.array_equal(Y[:, q], yo)
                continue
            bound = abs(coef[0]) * np.abs(xs[q])
            v = np.abs(xs[q])
            for a in coef[1:]:
                v = absL @ v
                bound = bound + abs(a) * v
            ratio = np.abs(Y[:, q] - yo) / (256 * EPS * bound[pos])
            worst = max(worst, float(ratio.max()))
        print(f"{kind} h={h} nrhs={nrhs} degree {deg}: max error / bound = {worst:.3f}", flush=True)
        assert worst <= 1.0


def _biharm_setup(kind, h, c0=1.0):
    params, d = ((1.0,), 2) if kind == "circle" else ((1.0,), 3)
    lb = G.lib_band(kind, params, d, h, 3)
    _, cp, _ = lb.export()
    cpa = cp[:lb.n_active]
    if kind == "circle":
        u, lam = inputs.circle_sin(cpa), 1.0
    else:
        u, lam = inputs.sphere_y4(cpa, 2), 20.0
    op = cpm.Operator(lb, np.sqrt(c0))
    f = torch.tensor((c0 + lam * lam) * u, dtype=torch.float64, device=DEV)
    return lb, op, f, u


def test_shifted_biharmonic_solve_matches_direct():
    c0, h = 1.0, 0.1
    lb, op, f, uex = _biharm_setup("sphere", h, c0)
    ob, E, O, A, P = G.oracle("sphere", (1.0,), 3, h, 3, 1.0)
    keys, pos = G.mapping(lb, ob)
    inv = np.argsort(pos)
    M = gridfunc.poly_matrix(gridfunc.laplace_beltrami(A, 1.0), [c0, 0.0, 1.0])
    fo = f.cpu().numpy()[inv]
    uo = spla.spsolve(M.tocsc(), fo)
    pc = cpm.Precond(op, kind="oras", n_parts=8, overlap=2.0, precision="fp64")
    its = {}
    for power in (1, 2):
        u, st = cpm.solve(op, f, pc=pc, rtol=1e-10, max_it=20000, poly=(c0, 0.0, 1.0), pc_power=power)
        its[power] = st["iterations"]
        assert st["converged"], st
        ul = u.cpu().numpy()[inv]
        res = np.linalg.norm(fo - M @ ul) / np.linalg.norm(fo)
        err = np.abs(ul - uo).max() / np.abs(uo).max()
        print(f"sphere h={h}: pc_power={power}: {st['iterations']} iterations, residual {res:.2e}, "
              f"|u - u_direct| {err:.2e}", flush=True)
        assert res <= 1e-10 * 1.05
        assert err <= 1e-7
    u, st = cpm.solve(op, f, rtol=1e-10, max_it=20000, poly=(c0, 0.0, 1.0))
    print(f"sphere h={h}: no preconditioner: {st['iterations']} iterations, converged={st['converged']}",
          flush=True)


@pytest.mark.parametrize("kind,hs,rtol", [("circle", (0.1, 0.05, 0.025), 1e-7), ("sphere", (0.1, 0.05), 1e-8)])
def test_shifted_biharmonic_second_order(kind, hs, rtol):
    errs = []
    for h in hs:
        lb, op, f, uex = _biharm_setup(kind, h)
        nparts = 4 if kind == "circle" else 8
        pc = cpm.Precond(op, kind="oras", n_parts=nparts, overlap=2.0, precision="fp64", coarse="first")
        u, st = cpm.solve(op, f, pc=pc, rtol=rtol, max_it=40000, poly=(1.0, 0.0, 1.0), pc_power=2, restart=60,
                          stagnation_cycles=400)
        assert st["converged"], st
        e = np.abs(u.cpu().numpy() - uex).max() / np.abs(uex).max()
        print(f"{kind} h={h} N_A={lb.n_active}: {st['iterations']} iterations, error {e:.3e}", flush=True)
        errs.append(e)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print(kind, "rates", rates, flush=True)
    assert (rates > 1.6).all(), (errs, rates)


def test_batched_biharmonic_equals_solo():
    ops, pcs, fs = [], [], []
    for kind, params, h in (("sphere", (1.0,), 0.05), ("torus", (1.0, 0.4), 0.05)):
        lb = G.lib_band(kind, params, 3, h, 3)
        op = cpm.Operator(lb, 1.0)
        ops.append(op)
        pcs.append(cpm.Precond(op, kind="oras", n_parts=8, overlap=2.0, precision="fp64", coarse="first"))
        fs.append(torch.tensor(G.field(lb.active_keys, 91), dtype=torch.float64, device=DEV))
    b = cpm.Batch(ops, pcs, [1, 1])
    kw = dict(rtol=1e-6, max_it=40000, poly=(1.0, 0.0, 1.0), pc_power=2, restart=60, stagnation_cycles=400)
    us, stats = b.solve(fs, **kw)
    assert all(s["converged"] for s in stats), stats
    for k in range(2):
        u1, st1 = cpm.solve(ops[k], fs[k], pc=pcs[k], **kw)
        assert torch.equal(us[k], u1), k
        assert st1["iterations"] == stats[k]["iterations"]
    # the batch's plain operator is untouched by the polynomial solve
    ys = b.apply(fs)
    for k in range(2):
        assert torch.equal(ys[k], ops[k].apply(fs[k]))


def test_poly_rejects_bad_options():
    lb = G.lib_band("sphere", (1.0,), 3, 0.1, 3)
    op = cpm.Operator(lb, 1.0)
    f = torch.ones(lb.n_active, dtype=torch.float64, device=DEV)
    for kw in (dict(poly=(1.0, 0.0, 1.0), transpose=True), dict(poly=(1.0, 0.0, 1.0), use_graph=True),
               dict(poly=(0.0, 0.0)), dict(poly=(1.0, float("nan"))), dict(pc_power=7)):
        with pytest.raises(_capi.CpmError):
            cpm.solve(op, f, raise_on_fail=True, **kw)
    with pytest.raises(_capi.CpmError):
        op.poly_apply([1.0, float("inf")], f)


def test_biharmonic_inner_solve_preconditioner_flat_in_h():
    """Each preconditioner application as an inner FGMRES solve of A(sqrt(c0)) (ORAS,
    to 1e-3), applied twice: A(sqrt(c0))^-2 is spectrally equivalent to (c0 + L^2)^-1, so
    the outer iteration count stays small and flat from h = 0.1 to 0.05 (the oracle's
    exact A(1)^-2 preconditioner gives 6 and 5 GMRES iterations there); the solutions
    equal those of the squared-ORAS solves to the tolerance and keep the manufactured
    errors."""
    its = []
    for h, expect in ((0.1, 7.117e-01), (0.05, 1.762e-01)):
        lb, op, f, uex = _biharm_setup("sphere", h)
        pc = cpm.Precond(op, kind="oras", n_parts=8, overlap=2.0, precision="fp64", coarse="first")
        u, st = cpm.solve(op, f, pc=pc, rtol=1e-8, max_it=2000, poly=(1.0, 0.0, 1.0), pc_power=2,
                          pc_inner_rtol=1e-3, pc_inner_max_it=60)
        assert st["converged"], st
        e = np.abs(u.cpu().numpy() - uex).max() / np.abs(uex).max()
        print(f"sphere h={h}: inner-solve preconditioner, {st['iterations']} outer iterations, "
              f"{st['ms_total']:.1f} ms, error {e:.4e}", flush=True)
        assert abs(e - expect) <= 1e-3 * expect
        its.append(st["iterations"])
    assert max(its) <= 30, its
