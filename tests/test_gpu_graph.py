"""Graph-captured restart cycles: a solve that replays each cycle as one
captured graph must equal the eager solve bit for bit (same kernels, same
arguments; steps after convergence are gated into no-ops). Every replay is
checked: the graph is replayed many times per solve and reused across solves,
with eager library work and synchronisations in between.
"""
import numpy as np
import pytest
import torch

from paper_2110_06322_amd import cpm, inputs, workloads
from paper_2110_06322_amd._capi import CpmError
from tests import gpu_cases as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sphere():
    G.ensure_built()
    b = cpm.Band("sphere", (1.0,), 3, 0.05, 3)
    op = cpm.Operator(b, 1.0)
    f = torch.tensor(21.0 * inputs.sphere_y4(b.export()[1][:b.n_active], 2), dtype=torch.float64, device="cuda")
    pcs = {p: cpm.Precond(op, kind="oras", n_parts=16, overlap=2.0, precision=p) for p in ("fp64", "fp32")}
    return b, op, f, pcs


@pytest.mark.parametrize("mode,prec", [("fp64", "fp64"), ("mixed", "fp32")])
def test_graph_solve_equals_eager(sphere, mode, prec):
    b, op, f, pcs = sphere
    pc = pcs[prec]
    u0, s0 = cpm.solve(op, f, pc=pc, rtol=1e-9, mode=mode, max_it=3000)
    assert s0["converged"]
    for rep in range(3):
        u1, s1 = cpm.solve(op, f, pc=pc, rtol=1e-9, mode=mode, max_it=3000, use_graph=True)
        torch.cuda.synchronize()
        assert s1["converged"] and s1["iterations"] == s0["iterations"], (rep, s0, s1)
        assert torch.equal(u1, u0), rep
        # eager work between replays
        y = op.apply(u1)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()


def test_graph_unpreconditioned_and_short_restart(sphere):
    b, op, f, _ = sphere
    u0, s0 = cpm.solve(op, f, rtol=1e-6, restart=7, max_it=4000)
    u1, s1 = cpm.solve(op, f, rtol=1e-6, restart=7, max_it=4000, use_graph=True)
    assert s0["iterations"] == s1["iterations"]
    assert torch.equal(u0, u1)


def test_graph_transposed_solve(sphere):
    b, op, f, _ = sphere
    pcT = cpm.Precond(op, kind="ras", n_parts=16, transpose=True)
    u0, s0 = cpm.solve(op, f, pc=pcT, rtol=1e-9, transpose=True)
    u1, s1 = cpm.solve(op, f, pc=pcT, rtol=1e-9, transpose=True, use_graph=True)
    assert s0["converged"] and s0["iterations"] == s1["iterations"]
    assert torch.equal(u0, u1)


def test_graph_batch_equals_eager():
    G.ensure_built()
    insts = workloads.batched(n_each=1, hs=(0.05,), nrhs=4, n_sub_range=(4, 8))
    bt = cpm.Batch([i.op for i in insts], [i.pc for i in insts], [4] * len(insts))
    us0, st0 = bt.solve([i.f for i in insts], rtol=1e-8, mode="mixed", max_it=3000)
    for _ in range(2):
        us1, st1 = bt.solve([i.f for i in insts], rtol=1e-8, mode="mixed", max_it=3000, use_graph=True)
        torch.cuda.synchronize()
        assert [s["iterations"] for s in st0] == [s["iterations"] for s in st1]
        for a, c in zip(us0, us1):
            assert torch.equal(a, c)


def test_graph_rejects_profile(sphere):
    b, op, f, pcs = sphere
    with pytest.raises(CpmError):
        cpm.solve(op, f, pc=pcs["fp64"], rtol=1e-8, use_graph=True, profile=True)


def test_graph_packet_layout_equals_eager(sphere):
    """Distance-ordered factors (packet subdomain solves) inside captured cycles."""
    b, op, f, _ = sphere
    pc = cpm.Precond(op, kind="oras", n_parts=16, overlap=2.0, precision="fp32", ordering="distance")
    u0, s0 = cpm.solve(op, f, pc=pc, rtol=1e-9, mode="mixed", max_it=3000)
    assert s0["converged"]
    for _ in range(2):
        u1, s1 = cpm.solve(op, f, pc=pc, rtol=1e-9, mode="mixed", max_it=3000, use_graph=True)
        torch.cuda.synchronize()
        assert s1["iterations"] == s0["iterations"]
        assert torch.equal(u1, u0)
        y = op.apply(u1)
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
