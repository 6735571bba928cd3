"""GPU parity of the matrix-free operator kernels against the oracle's assembled CSR.

Tolerance (per element, FP64): |y - y_oracle| <= 256 eps * s_i, with
s = (c + 2d/h^2)|x| + h^-2 O |E| |x| the sum of the magnitudes of the terms the
two sides combine (a forward-error bound for any summation order; the factor
covers the 64-term contraction, weight evaluation and the stencil sum).
"""
import numpy as np
import pytest
import torch

from paper_2110_06322_amd import cpm
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu
DEV = "cuda"
C_SHIFT = 1.7


@pytest.fixture(scope="module", autouse=True)
def _built():
    G.ensure_built()
    print("gpu operator tests: device count", cpm.device_count(), flush=True)


@pytest.mark.parametrize("case", G.cases(), ids=lambda c: f"{c[0]}-h{c[3]}-p{c[4]}")
def test_apply_extend_transpose_parity(case):
    kind, params, d, h, p = case
    print("case", case, flush=True)
    lb = G.lib_band(kind, params, d, h, p)
    ob, E, O, A, P = G.oracle(kind, params, d, h, p, C_SHIFT)
    keys, pos = G.mapping(lb, ob)
    op = cpm.Operator(lb, C_SHIFT)
    xo = G.field(ob.active_keys, 11)
    x = torch.tensor(G.field(keys, 11), dtype=torch.float64, device=DEV)
    # A x
    y = op.apply(x).cpu().numpy()
    yo = A @ xo
    bound = G.apply_bound(ob, E, O, C_SHIFT, xo)
    assert (np.abs(y - yo[pos]) <= 256 * G.EPS * bound[pos]).all(), np.max(np.abs(y - yo[pos]) / bound[pos])
    # determinism: bitwise identical on a second launch
    assert np.array_equal(op.apply(x).cpu().numpy(), y)
    # E x over Sigma_A u Sigma_G
    akeys, apos = G.all_mapping(lb, ob)
    v = op.extend(x).cpu().numpy()
    vo = E @ xo
    vb = abs(E) @ np.abs(xo)
    assert (np.abs(v - vo[apos]) <= 64 * G.EPS * vb[apos]).all()
    # A^T x
    yt = op.apply_T(x).cpu().numpy()
    yto = A.T @ xo
    h2 = h * h
    bt = (C_SHIFT + 2 * d / h2) * np.abs(xo) + (abs(E).T @ (O.T @ np.abs(xo))) / h2
    assert (np.abs(yt - yto[pos]) <= 256 * G.EPS * bt[pos]).all()
    # <A x, z> = <x, A^T z> on the device results
    z = torch.tensor(G.field(keys, 12), dtype=torch.float64, device=DEV)
    lhs = float(torch.dot(op.apply(x), z))
    rhs = float(torch.dot(x, op.apply_T(z)))
    assert abs(lhs - rhs) <= 1e-12 * float(torch.dot(op.apply(x).abs(), z.abs()))


@pytest.mark.parametrize("nrhs", [2, 4])
def test_apply_multi_rhs_interleaved(nrhs):
    kind, params, d, h, p = "torus", (1.0, 0.4), 3, 0.05, 3
    lb = G.lib_band(kind, params, d, h, p)
    ob, E, O, A, P = G.oracle(kind, params, d, h, p, C_SHIFT)
    keys, pos = G.mapping(lb, ob)
    op = cpm.Operator(lb, C_SHIFT)
    X = np.stack([G.field(keys, 20 + r) for r in range(nrhs)], axis=1)
    x = torch.tensor(X.copy(), dtype=torch.float64, device=DEV).reshape(-1)
    y = op.apply(x, nrhs=nrhs).cpu().numpy().reshape(-1, nrhs)
    yt = op.apply_T(x, nrhs=nrhs).cpu().numpy().reshape(-1, nrhs)
    for r in range(nrhs):
        xo = G.field(ob.active_keys, 20 + r)
        bound = G.apply_bound(ob, E, O, C_SHIFT, xo)
        assert (np.abs(y[:, r] - (A @ xo)[pos]) <= 256 * G.EPS * bound[pos]).all()
        assert np.abs(yt[:, r] - (A.T @ xo)[pos]).max() <= 1e-12 * np.abs(A.T @ xo).max()
        # each column equals the single right-hand-side apply bit for bit
        y1 = op.apply(torch.tensor(X[:, r].copy(), dtype=torch.float64, device=DEV)).cpu().numpy()
        assert np.array_equal(y1, y[:, r])


def test_shift_update_and_constant_vector():
    lb = G.lib_band("sphere", (1.0,), 3, 0.1, 3)
    op = cpm.Operator(lb, 1.0)
    one = torch.ones(lb.n_active, dtype=torch.float64, device=DEV)
    for c in (1.0, 3.25, 1e4):
        op.set_shift(c)
        y = op.apply(one)
        diag = c + 6 / 0.01
        assert float((y - c).abs().max()) <= 64 * G.EPS * 2 * diag


def _force_apply(path, variant):
    import json
    c = json.loads(path.read_text())
    keys = [k for k in c if k.startswith("apply|")]
    assert keys
    for k in keys:
        c[k] = [variant]
    path.write_text(json.dumps(c))


@pytest.mark.parametrize("case", G.cases(), ids=lambda c: f"{c[0]}-h{c[3]}-p{c[4]}")
def test_two_pass_apply_equals_fused(case, tmp_path):
    """The two-pass apply (extension rows of every band node once into a scratch vector, then
    the stencil) gives the fused kernel's bits: the same extension-row arithmetic and the same
    order of the neighbour sum. The fused kernel is the one checked against the oracle above."""
    kind, params, d, h, p = case
    lb = G.lib_band(kind, params, d, h, p)
    op = cpm.Operator(lb, C_SHIFT)
    x = torch.tensor(G.field(lb.active_keys, 11), dtype=torch.float64, device=DEV)
    cache = tmp_path / "tune.json"
    cpm.autotune(op, None, cache=cache)
    outs = {}
    for v in (0, 2):
        _force_apply(cache, v)
        r = cpm.autotune(op, None, cache=cache)
        assert r["apply_variant"] == v and r["from_cache"] == 1
        outs[v] = op.apply(x)
    assert torch.equal(outs[0], outs[2])


@pytest.mark.parametrize("case", [("sphere", (1.0,), 3, 0.05, 3), ("torus", (1.0, 0.4), 3, 0.05, 3),
                                  ("sphere", (1.0,), 3, 0.1, 2)], ids=lambda c: f"{c[0]}-h{c[3]}-p{c[4]}")
def test_fallback_tiles_equal_fused_and_oracle(case):
    """A 16 KiB LDS budget sends the tiles whose footprint does not fit to the global-memory
    kernel (k_apply_fallback): its results equal the fused kernels' bit for bit (same
    contraction and stencil order) for 1, 2 and 4 right-hand sides, and the oracle's within
    the apply bar."""
    kind, params, d, h, p = case
    lb = G.lib_band(kind, params, d, h, p)
    ob, E, O, A, P = G.oracle(kind, params, d, h, p, C_SHIFT)
    keys, pos = G.mapping(lb, ob)
    op = cpm.Operator(lb, C_SHIFT)
    small = cpm.Operator(lb, C_SHIFT, lds_bytes=16384)
    inf, infs = op.info, small.info
    print(f"{kind} h={h}: tiles {inf['n_tiles']}, fallback tiles {inf['n_fallback_tiles']} at 64 KiB, "
          f"{infs['n_fallback_tiles']} at 16 KiB", flush=True)
    assert infs["n_tiles"] == inf["n_tiles"] and infs["n_fallback_tiles"] > inf["n_fallback_tiles"]
    assert infs["apply_lds_bytes"] == 16384 and inf["apply_lds_bytes"] == 65536
    for nrhs in (1, 2, 4):
        xs = [G.field(ob.active_keys, 70 + q) for q in range(nrhs)]
        X = torch.tensor(np.stack([x[pos] for x in xs], axis=1).ravel(), dtype=torch.float64, device=DEV)
        y_small = small.apply(X, nrhs=nrhs)
        assert torch.equal(y_small, op.apply(X, nrhs=nrhs)), nrhs
        Y = y_small.cpu().numpy().reshape(-1, nrhs)
        for q in range(nrhs):
            bound = G.apply_bound(ob, E, O, C_SHIFT, xs[q])
            assert (np.abs(Y[:, q] - (A @ xs[q])[pos]) <= 256 * G.EPS * bound[pos]).all()
