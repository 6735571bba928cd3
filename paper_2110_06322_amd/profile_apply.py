"""Short, profiler-friendly driver: a fixed number of operator applies (or,
with a fourth argument, ORAS preconditioner applies with that local row order
and FP32 factors, 64 subdomains, overlap 2h, `transpose` transpose applies, or
`order4` applies of the fourth-order operator on a band of reach 2, with the
interpolation degree as a fifth argument, default 3; or `solve2`: `reps`
mixed solves to 1e-8 of f = 21 Y4 with the two-level coarse-first FP32 ORAS,
distance order, the number of subdomains as the fifth argument, default 64) on
one workload and a
device-to-device copy of known size (the copy calibrates the hardware byte
counters against a kernel whose traffic is exactly known). Applies rotate
through four input/output pairs, as the benchmark's do.

Usage: python -m paper_2110_06322_amd.profile_apply [sphere|torus] [h] [reps] [rcm|distance|transpose|order4|solve2] [p|parts]
"""
from __future__ import annotations

import sys

import torch

from . import cpm, inputs


def main():
    kind = sys.argv[1] if len(sys.argv) > 1 else "sphere"
    h = float(sys.argv[2]) if len(sys.argv) > 2 else 0.02
    reps = int(sys.argv[3]) if len(sys.argv) > 3 else 20
    params = (1.0,) if kind == "sphere" else (1.0, 0.4)
    mode = sys.argv[4] if len(sys.argv) > 4 else None
    if mode == "order4":
        p = int(sys.argv[5]) if len(sys.argv) > 5 else 3
        band = cpm.Band(kind, params, 3, h, p, reach=2)
        op = cpm.Operator(band, 1.0, order=4)
    else:
        band = cpm.Band(kind, params, 3, h, 3)
        op = cpm.Operator(band, 1.0)
    xs = [torch.tensor(inputs.normal(10 + i, 0, band.active_keys), dtype=torch.float64, device="cuda")
          for i in range(4)]
    ys = [torch.empty_like(x) for x in xs]
    if mode in ("rcm", "distance"):
        pc = cpm.Precond(op, kind="oras", n_parts=64, overlap=2.0, precision="fp32", ordering=mode)
        cpm.autotune(op, pc)
        for r in range(reps):
            pc.apply(xs[r % 4], out=ys[r % 4])
    elif mode == "solve2":
        parts = int(sys.argv[5]) if len(sys.argv) > 5 else 64
        _, cp, _ = band.export()
        f = torch.tensor(21.0 * inputs.sphere_y4(cp[:band.n_active], 2), dtype=torch.float64, device="cuda")
        pc = cpm.Precond(op, kind="oras", n_parts=parts, overlap=2.0, precision="fp32", ordering="distance",
                         coarse="first")
        cpm.autotune(op, pc)
        for r in range(reps):
            u, st = cpm.solve(op, f, pc=pc, rtol=1e-8, mode="mixed", max_it=20000)
            print(f"solve {r}: {st['iterations']} iterations, {st['ms_total']:.2f} ms", flush=True)
    elif mode == "transpose":
        for r in range(reps):
            op.apply_T(xs[r % 4], out=ys[r % 4])
    elif mode == "order4":
        for r in range(reps):
            op.apply(xs[r % 4], out=ys[r % 4])
    else:
        cpm.autotune(op, None)
        for r in range(reps):
            op.apply(xs[r % 4], out=ys[r % 4])
    a = torch.zeros(64 * 1024 * 1024 // 8, dtype=torch.float64, device="cuda")  # 64 MiB
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"{kind} h={h}: N_A={band.n_active} N_G={band.n_ghost} applies={reps}; copy 64 MiB x4", flush=True)


if __name__ == "__main__":
    main()
