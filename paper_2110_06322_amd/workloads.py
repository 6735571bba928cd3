"""The synthetic workloads the library is exercised on, built through the C ABI.

Each builder returns plain objects (bands, operators, preconditioners,
right-hand sides on the GPU). Inputs come from the seeded generators of
`inputs`; nothing here evaluates the method itself.

  circle   : 2-D unit circle, h = 0.05 on [-2,2]^2, p = 2, c = 1, f = 2 sin(theta)
  sphere   : unit sphere, h = 0.02 on [-2,2]^3, p = 3, c = 1, f = 21 Y_4 (seed 2),
             (O)RAS with 64 boxes and overlap 2h
  batched  : 48 surfaces (16 spheres, 16 ellipsoids with semi-axes ~U[0.6,1.4],
             16 tori R = 1, r ~ U[0.3,0.5]) at h cyclic over {0.04, 0.02, 0.01},
             p = 3, c ~ U[0.5,10] per surface, 4 N(0,1) right-hand sides each,
             grid box [-2,2]^3 (wider only where a coarse band needs it),
             clamp(2^round(log2(N_A/2048)), 32, 512) subdomains, FP32 ORAS
  adjoint  : torus R = 1, r = 0.4, h = 0.01, p = 3, c = 1, f and the target from
             seeded toroidal/poloidal modes
  grayscott: torus R = 1, r = 0.4, h = 0.005, p = 3 (see gray_scott.py)
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

from . import cpm, inputs


@dataclass
class Instance:
    band: cpm.Band
    op: cpm.Operator
    pc: cpm.Precond | None
    f: torch.Tensor          # [N_A * nrhs] interleaved
    nrhs: int
    meta: dict = field(default_factory=dict)


def circle(device="cuda") -> Instance:
    b = cpm.Band("circle", (1.0,), 2, 0.05, 2)
    op = cpm.Operator(b, 1.0)
    _, cp, _ = b.export()
    f = torch.tensor(2.0 * inputs.circle_sin(cp[:b.n_active]), dtype=torch.float64, device=device)
    return Instance(b, op, None, f, 1, {"rtol": 1e-10})


def sphere(precision="fp64", kind="oras", h=0.02, n_parts=64, device="cuda") -> Instance:
    b = cpm.Band("sphere", (1.0,), 3, h, 3)
    op = cpm.Operator(b, 1.0)
    pc = cpm.Precond(op, kind=kind, n_parts=n_parts, overlap=2.0, precision=precision)
    _, cp, _ = b.export()
    f = torch.tensor(21.0 * inputs.sphere_y4(cp[:b.n_active], 2), dtype=torch.float64, device=device)
    return Instance(b, op, pc, f, 1, {"rtol": 1e-8})


# host threads for independent setups: the library's host code releases the GIL
# (ctypes) and each setup also runs its own OpenMP loops
SETUP_THREADS = 4


def preconditioners(ops, n_parts, precision="fp32", ordering="rcm", kind="oras", overlap=2.0,
                    threads=SETUP_THREADS, coarse="none"):
    """(O)RAS preconditioners for several operators, built concurrently, in order."""
    def one(args):
        op, ns = args
        return cpm.Precond(op, kind=kind, n_parts=ns, overlap=overlap, precision=precision, ordering=ordering,
                           coarse=coarse)
    with ThreadPoolExecutor(max(1, threads)) as ex:
        return list(ex.map(one, zip(ops, n_parts)))


def batched(n_each=16, hs=(0.04, 0.02, 0.01), nrhs=4, precision="fp32", kind="oras", seed=3,
            n_sub_range=(32, 512), device="cuda", ordering="rcm", threads=SETUP_THREADS) -> list[Instance]:
    specs = list(inputs.batch_instances(seed=seed, n_each=n_each, hs=hs))

    def one(item):
        i, spec = item
        box = inputs.domain_box(spec["kind"], spec["params"], 3, spec["h"], 3)
        b = cpm.Band(spec["kind"], spec["params"], 3, spec["h"], 3, lo=box[0], hi=box[1])
        op = cpm.Operator(b, spec["c"])
        ns = inputs.n_subdomains_for(b.n_active, *n_sub_range)
        pc = cpm.Precond(op, kind=kind, n_parts=ns, overlap=2.0, precision=precision, ordering=ordering)
        keys = b.active_keys
        F = np.stack([inputs.normal(seed * 1000 + i, r, keys) for r in range(nrhs)], axis=1)
        f = torch.tensor(np.ascontiguousarray(F).reshape(-1), dtype=torch.float64, device=device)
        return Instance(b, op, pc, f, nrhs, dict(spec, n_sub=ns, box=box))

    # largest first, so that the long setups start early; results keep the spec order
    order = sorted(range(len(specs)), key=lambda i: specs[i]["h"])
    with ThreadPoolExecutor(max(1, threads)) as ex:
        built = dict(zip(order, ex.map(one, [(i, specs[i]) for i in order])))
    return [built[i] for i in range(len(specs))]


def adjoint_torus(h=0.01, n_parts=128, device="cuda"):
    b = cpm.Band("torus", (1.0, 0.4), 3, h, 3)
    op = cpm.Operator(b, 1.0)
    _, cp, _ = b.export()
    cpa = cp[:b.n_active]
    f = torch.tensor(inputs.torus_modes(cpa, 1.0, seed=41), dtype=torch.float64, device=device)
    ut = torch.tensor(inputs.torus_modes(cpa, 1.0, seed=42), dtype=torch.float64, device=device)
    pc = cpm.Precond(op, kind="ras", n_parts=n_parts)
    pcT = cpm.Precond(op, kind="ras", n_parts=n_parts, transpose=True)
    return b, op, pc, pcT, f, ut
