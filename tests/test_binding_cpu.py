"""The Python binding refuses bad vectors before any library call (CPU only).

Every device pointer handed to the C ABI goes through cpm.check_vec (tensor,
float64, contiguous, exact element count, device), outputs are checked not to
overlap inputs, and per-instance lists must have one entry per instance. These
checks run before the library is reached, so they can be exercised here with
CPU tensors and stand-in objects: a wrong size raises ValueError instead of
letting a kernel read or write past the end of a buffer.
"""
import types

import pytest
import torch

from paper_2110_06322_amd import cpm


def test_check_vec_refusals():
    good = torch.zeros(12, dtype=torch.float64)
    with pytest.raises(TypeError):
        cpm.check_vec([0.0] * 12, 12, "x")
    with pytest.raises(ValueError, match="float64"):
        cpm.check_vec(good.float(), 12, "x")
    with pytest.raises(ValueError, match="contiguous"):
        cpm.check_vec(torch.zeros(24, dtype=torch.float64)[::2], 12, "x")
    with pytest.raises(ValueError, match="expected 48 elements"):
        cpm.check_vec(good, 48, "x")      # an N_A-sized vector passed with nrhs = 4
    assert cpm.check_vec(good, 12, "x") is good
    with pytest.raises(ValueError, match="device"):
        cpm.check_vec(good, 12, "x", on_device=True)      # right size, but host memory


def test_check_nrhs_and_overlap():
    for r in (1, 2, 4):
        assert cpm.check_nrhs(r) == r
    for r in (0, 3, 8, -1):
        with pytest.raises(ValueError):
            cpm.check_nrhs(r)
    base = torch.zeros(20, dtype=torch.float64)
    cpm.check_disjoint(base[:10], base[10:], "a and b")
    with pytest.raises(ValueError, match="overlap"):
        cpm.check_disjoint(base[:10], base[5:15], "a and b")
    with pytest.raises(ValueError, match="overlap"):
        cpm.check_disjoint(base, base, "a and b")


def _fake_operator(n):
    return types.SimpleNamespace(n_active=n, _h=None)


def test_operator_methods_refuse_wrong_sizes_before_the_library():
    op = cpm.Operator.__new__(cpm.Operator)
    op.n_active, op._h = 10, None
    op.band = types.SimpleNamespace(n_active=10, n_ghost=3)
    x = torch.zeros(10, dtype=torch.float64)
    with pytest.raises(ValueError, match="expected 40 elements"):
        op.apply(x, nrhs=4)
    with pytest.raises(ValueError, match="expected 10 elements"):
        op.apply_T(torch.zeros(9, dtype=torch.float64))
    with pytest.raises(ValueError, match="out: expected 10 elements"):
        op.apply(x, out=torch.zeros(11, dtype=torch.float64))
    with pytest.raises(ValueError, match="nrhs"):
        op.apply(x, nrhs=3)
    with pytest.raises(ValueError, match="out: expected 13 elements"):
        op.extend(x, out=torch.zeros(10, dtype=torch.float64))
    with pytest.raises(ValueError, match="expected 10 elements"):
        op.shift_gradient(torch.zeros(10, dtype=torch.float64), torch.zeros(8, dtype=torch.float64))
    with pytest.raises(ValueError, match="device"):
        op.apply(x)   # right size on the host: refused, never passed on
    op._h = None


def test_solve_and_precond_refuse_wrong_sizes():
    op = _fake_operator(6)
    with pytest.raises(ValueError, match="f: expected 24 elements"):
        cpm.solve(op, torch.zeros(6, dtype=torch.float64), nrhs=4)
    with pytest.raises(ValueError, match="u: expected 6 elements"):
        cpm.solve(op, torch.zeros(6, dtype=torch.float64), u=torch.zeros(5, dtype=torch.float64))
    pc = cpm.Precond.__new__(cpm.Precond)
    pc.op, pc._h = op, None
    with pytest.raises(ValueError, match="r: expected 12 elements"):
        pc.apply(torch.zeros(6, dtype=torch.float64), nrhs=2)


def test_batch_refuses_wrong_counts_and_sizes():
    b = cpm.Batch.__new__(cpm.Batch)
    b._ops = [_fake_operator(5), _fake_operator(7)]
    b._pcs = [None, None]
    b.nrhs = [1, 2]
    b.sizes = [5, 14]
    b._h = None
    v5, v14 = torch.zeros(5, dtype=torch.float64), torch.zeros(14, dtype=torch.float64)
    with pytest.raises(ValueError, match="fs: expected 2 entries"):
        b.solve([v5])
    with pytest.raises(ValueError, match=r"fs\[1\]: expected 14 elements"):
        b.solve([v5, torch.zeros(7, dtype=torch.float64)])
    with pytest.raises(ValueError, match="us: expected 2 entries"):
        b.solve([v5, v14], us=[v5, v14, v5])
    with pytest.raises(ValueError, match="xs: expected 2 entries"):
        b.apply([v5, v14, v5])
    with pytest.raises(ValueError, match=r"ys\[0\]: expected 5 elements"):
        b.apply([v5, v14], ys=[v14, v14])
    b._h = None
