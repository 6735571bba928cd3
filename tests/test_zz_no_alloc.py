"""The allocation-free transpose apply (cpm_apply_T_noalloc) against cpm_apply_T.

Called through the C ABI on the same inputs, twice in a row on one GPU (the
second time on a smaller band, so the static scratch array still holds the
first call's larger contents), and with several right-hand sides: results
equal the allocating entry point's bit for bit, since both run the same
kernels on the same data. Sizes beyond the static array are refused.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2110_06322_amd import _capi, cpm
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _raw(op, x, y, nrhs):
    s = torch.cuda.current_stream()
    return _capi.lib().cpm_apply_T_noalloc(op._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nrhs,
                                           C.c_void_p(s.cuda_stream))


@pytest.mark.parametrize("nrhs", [1, 4])
def test_noalloc_transpose_equals_allocating_entry_point(nrhs):
    G.ensure_built()
    cases = [("torus", (1.0, 0.4), 3, 0.05, 3), ("sphere", (1.0,), 3, 0.1, 3)]   # second call: smaller band
    sizes = []
    for k, (kind, params, d, h, p) in enumerate(cases):
        lb = G.lib_band(kind, params, d, h, p)
        sizes.append(lb.n_active + lb.n_ghost)
        op = cpm.Operator(lb, 1.3)
        X = np.stack([G.field(lb.active_keys, 40 + k + 10 * r) for r in range(nrhs)], axis=1)
        x = torch.tensor(X.reshape(-1).copy(), dtype=torch.float64, device=DEV)
        y0 = op.apply_T(x, nrhs=nrhs)
        y1 = torch.full_like(x, float("nan"))
        assert _raw(op, x, y1, nrhs) == _capi.CPM_OK, _capi.lib().cpm_last_error()
        torch.cuda.synchronize()
        print(f"call {k}: {kind} h={h} N_A+N_G={sizes[-1]} nrhs={nrhs}", flush=True)
        assert torch.equal(y0, y1)
        # through the binding as well
        y2 = op.apply_T_noalloc(x, out=torch.empty_like(x), nrhs=nrhs)
        assert torch.equal(y0, y2)
    assert sizes[1] < sizes[0]


def test_noalloc_transpose_refuses_oversize():
    G.ensure_built()
    lb = G.lib_band("torus", (1.0, 0.4), 3, 0.01, 3)
    n = lb.n_active + lb.n_ghost
    assert n * 4 > (1 << 22) >= n
    op = cpm.Operator(lb, 1.0)
    x = torch.zeros(lb.n_active * 4, dtype=torch.float64, device=DEV)
    y = torch.empty_like(x)
    assert _raw(op, x, y, 4) == 1   # CPM_ERR_ARG, nothing launched
    assert b"exceeds the static scratch" in _capi.lib().cpm_last_error()
    x1 = torch.tensor(G.field(lb.active_keys, 50), dtype=torch.float64, device=DEV)
    y1 = torch.empty_like(x1)
    assert _raw(op, x1, y1, 1) == _capi.CPM_OK
    assert torch.equal(y1, op.apply_T(x1))
