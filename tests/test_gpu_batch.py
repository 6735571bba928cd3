"""Batched solves: uneven surfaces, shifts, subdomain counts and four right-hand
sides advanced together in shared launches. Bar: every system of the batch
equals its solo solve bit for bit (the batched kernels do the same arithmetic
per system), and true residuals recomputed by the oracle meet the tolerance.
"""
import numpy as np
import pytest
import torch

from paper_2110_06322_amd import cpm, workloads
from tests import gpu_cases as G
from tests import oracle_cases as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small_batch():
    G.ensure_built()
    # 2 of each surface kind at h = 0.05 and 0.04 (the batched workload's recipe, coarser)
    return workloads.batched(n_each=2, hs=(0.05, 0.04), nrhs=4, n_sub_range=(4, 16))


def test_batch_apply_equals_single_applies(small_batch):
    b = cpm.Batch([i.op for i in small_batch], None, [4] * len(small_batch))
    ys = b.apply([i.f for i in small_batch])
    for inst, y in zip(small_batch, ys):
        y1 = inst.op.apply(inst.f, nrhs=4)
        assert torch.equal(y, y1)


def test_batch_mixed_solve_equals_solo_and_meets_tolerance(small_batch):
    insts = small_batch
    b = cpm.Batch([i.op for i in insts], [i.pc for i in insts], [4] * len(insts))
    us, stats = b.solve([i.f for i in insts], rtol=1e-8, mode="mixed", max_it=5000)
    assert all(s["converged"] for s in stats), stats
    print("iterations per system", [s["iterations"] for s in stats])
    for k, inst in enumerate(insts):
        u1, st1 = cpm.solve(inst.op, inst.f, pc=inst.pc, nrhs=4, rtol=1e-8, mode="mixed", max_it=5000)
        assert torch.equal(us[k], u1), k
    # true residual of one sphere, one ellipsoid, one torus, recomputed by the oracle
    for k in (0, 2, 4):
        inst = insts[k]
        spec = inst.meta
        box = tuple(tuple(v) for v in spec["box"])
        ob, E, O, A, P = C.matrices(spec["kind"], tuple(spec["params"]), 3, spec["h"], 3, spec["c"], box)
        keys, pos = G.mapping(inst.band, ob)
        inv = np.argsort(pos)
        U = us[k].cpu().numpy().reshape(-1, 4)
        F = inst.f.cpu().numpy().reshape(-1, 4)
        for r in range(4):
            res = np.linalg.norm(F[inv, r] - A @ U[inv, r]) / np.linalg.norm(F[:, r])
            assert res <= 1e-8 * 1.01, (k, r, res)


def test_batch_autotune_keeps_results(small_batch, tmp_path):
    insts = small_batch
    b = cpm.Batch([i.op for i in insts], [i.pc for i in insts], [4] * len(insts))
    us0, st0 = b.solve([i.f for i in insts], rtol=1e-8, mode="mixed", max_it=5000)
    r = b.autotune(cache=tmp_path / "t.json")
    assert r["precond_ms"] > 0 and r["from_cache"] == 0
    assert b.autotune(cache=tmp_path / "t.json")["from_cache"] == 1
    us1, st1 = b.solve([i.f for i in insts], rtol=1e-8, mode="mixed", max_it=5000)
    for a, c in zip(us0, us1):
        assert torch.equal(a, c)


def test_batch_rejects_mixed_dimensions():
    G.ensure_built()
    b2 = cpm.Band("circle", (1.0,), 2, 0.1, 3)
    b3 = cpm.Band("sphere", (1.0,), 3, 0.1, 3)
    ops = [cpm.Operator(b2, 1.0), cpm.Operator(b3, 1.0)]
    with pytest.raises(Exception):
        cpm.Batch(ops, None, [1, 1])


def test_batch_packet_layout_equals_solo():
    """Distance-ordered factors (packet kernel) in a batch: each system equals its solo solve."""
    insts = workloads.batched(n_each=1, hs=(0.05,), nrhs=4, n_sub_range=(4, 8), ordering="distance")
    b = cpm.Batch([i.op for i in insts], [i.pc for i in insts], [4] * len(insts))
    assert b.autotune()["schwarz_variant"] in (2, 3)
    us, stats = b.solve([i.f for i in insts], rtol=1e-8, mode="mixed", max_it=5000)
    assert all(s["converged"] for s in stats), stats
    for k, inst in enumerate(insts):
        u1, st1 = cpm.solve(inst.op, inst.f, pc=inst.pc, nrhs=4, rtol=1e-8, mode="mixed", max_it=5000)
        assert torch.equal(us[k], u1), k


def test_batch_rejects_mixed_layouts():
    G.ensure_built()
    b = cpm.Band("sphere", (1.0,), 3, 0.1, 3)
    op = cpm.Operator(b, 1.0)
    pcs = [cpm.Precond(op, n_parts=4, ordering=o) for o in ("rcm", "distance")]
    with pytest.raises(Exception):
        cpm.Batch([op, op], pcs, [1, 1])


def test_batch_level_count_packets_equal_solo():
    """Distance-ordered factors with one right-hand side per system: the batch runs the
    packet subdomain solves in the level-count form (forced through the tuner cache; one
    LDS counter per sweep, no per-dependency polls); each system equals its solo solve,
    run with the polling form, bit for bit."""
    import json
    import tempfile
    insts = workloads.batched(n_each=1, hs=(0.05,), nrhs=1, n_sub_range=(4, 8), ordering="distance")
    b = cpm.Batch([i.op for i in insts], [i.pc for i in insts], [1] * len(insts))
    with tempfile.TemporaryDirectory() as d:
        cache = f"{d}/tune.json"
        b.autotune(cache=cache)
        tab = json.load(open(cache))
        assert any(k.startswith("batch-schwarz|") for k in tab), list(tab)
        for k in tab:
            if k.startswith("batch-schwarz|"):
                tab[k] = [4, 256, 1]
        json.dump(tab, open(cache, "w"))
        res = b.autotune(cache=cache)
        assert res["schwarz_variant"] == 4 and res["from_cache"] == 1, res
        us, stats = b.solve([i.f for i in insts], rtol=1e-8, mode="mixed", max_it=5000)
    assert all(s["converged"] for s in stats), stats
    for k, inst in enumerate(insts):
        u1, st1 = cpm.solve(inst.op, inst.f, pc=inst.pc, rtol=1e-8, mode="mixed", max_it=5000)
        assert torch.equal(us[k], u1), k
        assert st1["iterations"] == stats[k]["iterations"]
