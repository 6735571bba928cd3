"""Benchmark of the CPM hot path on one MI355X.

Headline workload (the largest configuration): the semi-implicit Gray-Scott
system on the torus R = 1, r = 0.4, grid h = 0.005 on [-2,2]^3, p = 3
(N_A = 3 643 824 active nodes), mu = (2e-5, 1e-5), F = 0.04, k = 0.06,
dt = 1, so each step solves (1/(mu_w dt) - Lap_S^h) w = rhs_w for both
species as one batch of two shifted systems with FP32 ORAS preconditioners
(1024 boxes, overlap 2h) inside FP64 FGMRES with iterative refinement to 1e-8.
One step = one Gray-Scott step (reaction right-hand side, two batched solves:
extension + stabilized operator applies, Schwarz subdomain solves, Krylov
core) followed by a burst of operator applies on that torus, rotating through
four input/output pairs so that repetitions read HBM rather than the 256 MB
last-level cache (HIP events on the apply's stream bracket the burst).

Reported: value = operator-apply throughput of the fused apply kernel on the
torus (active nodes per second); `roofline` for that kernel (algorithmic bytes
per active node = 8 (x) + 8 (y) + 8 d (1 + N_G/N_A) closest-point coordinates;
`traffic` = counter-measured HBM bytes per launch from the committed summary
while its sources are unchanged); `gray_scott` = mixed vs FP64 step time;
`solve` = unit sphere h = 0.02 ORAS-GMRES to 1e-8, mixed vs FP64, with each
solution's error against the CPU oracle's reference solve; `batched` = the
48-surface batch to 1e-8, mixed vs FP64; `apply_scaling` = the apply on the
torus h = 0.0025 (0.69 GB per apply) and on the sphere h = 0.02
(cache-resident); `apply_T` = the transpose apply on the torus h = 0.01;
`cpu_baseline` = the CPU oracle (CSR matvec on a bounded sample, and its
reference solve of the sphere system), rank 0 only.

The oracle runs in a child process that never touches the GPU (one thread,
started first so that it overlaps the GPU legs); its matvec timing starts
only after the GPU legs have finished, so nothing else competes for the host.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "CPM apply Gnodes/s (%HBM peak); ORAS-GMRES time to 1e-8, mixed vs FP64"


def _args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--apply-burst", type=int, default=20, help="torus applies timed per step")
    ap.add_argument("--tune-cache", default=None, help="JSON cache of the autotuner (default: tune afresh)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ordering", default="distance", help="local row order of the sphere solve leg")
    ap.add_argument("--gs-ordering", default="distance", help="local row order of the Gray-Scott step")
    ap.add_argument("--batched-ordering", default="rcm",
                    help="row order of the batched leg (rcm: fewer iterations win on mixed surfaces)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 48-surface batched leg")
    ap.add_argument("--no-scaling", action="store_true", help="skip the other apply workloads")
    ap.add_argument("--no-extensions", action="store_true",
                    help="skip the IMEX / two-level / biharmonic / fourth-order / open-surface timings")
    ap.add_argument("--oracle-worker", default=None, help=argparse.SUPPRESS)
    return ap.parse_args(argv)


# ---------------------------------------------------------------- CPU oracle (child process)
def oracle_worker(outdir):
    """Runs in a child process with one BLAS/OpenMP thread and no GPU. Writes
    ref.npz (the oracle's reference solution of the unit sphere h = 0.02 system)
    and ref.json, then waits for the file `go` before timing the CSR matvec
    sample, and writes cpu.json."""
    import numpy as np

    from oracle import band as OB, krylov, operator as OO, schwarz, surfaces as OS
    from paper_2110_06322_amd import inputs

    def log(msg):
        print(f"oracle: {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    h = 0.02
    bd = OB.build_band(OS.make_cp("sphere", (1.0,)), 3, h, 3, [-2.0] * 3, [2.0] * 3,
                       inputs.ruuth_merriman_gamma(3, 3, h))
    E = OO.assemble_E(bd)
    Om = OO.assemble_O(bd)
    A = OO.assemble_A(bd, 1.0, E, Om)
    P = OO.structural_pattern(bd, Om)
    A = OO.values_on_pattern(A, P)
    t_build = time.perf_counter() - t0
    log(f"sphere h=0.02 assembled in {t_build:.1f} s")
    f = 21.0 * inputs.sphere_y4(bd.cp_active, 2)
    t0 = time.perf_counter()
    S = schwarz.build_schwarz(A, P, bd.cp_active, bd.active_keys, h, 64, 2.0, kind="ras", subsolver="lu")
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    x, info = krylov.fgmres(A, f, M=S.apply, restart=30, rtol=1e-13, max_it=3000)
    t_solve = time.perf_counter() - t0
    log(f"reference solve {t_solve:.1f} s, {info['iters']} iterations")
    np.savez(os.path.join(outdir, "ref.npz"), keys=bd.active_keys, x=x)
    with open(os.path.join(outdir, "ref.json"), "w") as fh:
        json.dump({"seconds": round(t_solve, 2), "setup_seconds": round(t_setup, 2), "cores": 1,
                   "iterations": int(info["iters"]), "relres": float(info["relres"]),
                   "method": "oracle FGMRES(30), MGS, right-preconditioned by RAS with exact local LU "
                             "(64 boxes, overlap 2h), to 1e-13; unit sphere h=0.02, N_A=%d" % bd.n_active}, fh)
    # matvec sample: the torus of the headline workload at h = 0.02 (the oracle's band
    # construction visits every grid node, so the h = 0.005 band itself takes it tens of
    # minutes; rows have the same surface, degree and 3-D stencil structure)
    ht = 0.02
    tb = OB.build_band(OS.make_cp("torus", (1.0, 0.4)), 3, ht, 3, [-2.0] * 3, [2.0] * 3,
                       inputs.ruuth_merriman_gamma(3, 3, ht))
    At = OO.assemble_A(tb, 1.0)
    xt = inputs.normal(1, 0, tb.active_keys)
    log("torus h=0.02 assembled; waiting for the GPU legs to finish")
    go = os.path.join(outdir, "go")
    parent, waited = os.getppid(), 0.0
    while not os.path.exists(go):
        if os.getppid() != parent or waited > 3600:   # the benchmark has gone: give up quietly
            return
        time.sleep(0.5)
        waited += 0.5
    reps, t0 = 0, time.perf_counter()
    while True:
        At @ xt
        reps += 1
        el = time.perf_counter() - t0
        if el > 20.0:
            break
    with open(os.path.join(outdir, "cpu.json"), "w") as fh:
        json.dump({"value": round(tb.n_active * reps / el / 1e9, 5), "unit": "Gnodes/s", "cores": 1,
                   "kind": "oracle",
                   "sample": f"{reps} SciPy CSR matvecs in {el:.1f} s of the oracle's assembled FP64 operator on "
                             f"the torus R=1 r=0.4 at h=0.02 (N_A={tb.n_active}, p=3: the headline surface and row "
                             "structure at 1/16 of its nodes; the oracle's own band construction for h=0.005 "
                             "takes tens of minutes); one thread"}, fh)


def start_oracle():
    d = tempfile.mkdtemp(prefix="cpm_oracle_")
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="", ROCR_VISIBLE_DEVICES="")
    p = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker", d], env=env)
    return p, d


def finish_oracle(p, d, timeout=900):
    open(os.path.join(d, "go"), "w").close()
    try:
        p.wait(timeout=timeout)
    except subprocess.TimeoutExpired:
        p.kill()
        p.wait()
    out = {}
    for name in ("ref.json", "cpu.json"):
        f = os.path.join(d, name)
        if os.path.exists(f):
            out[name] = json.load(open(f))
    ref = os.path.join(d, "ref.npz")
    if os.path.exists(ref):
        import numpy as np
        z = np.load(ref)
        out["ref"] = (z["keys"], z["x"])
    return out


# ---------------------------------------------------------------- helpers
APPLY_SOURCES = ("apply.hip", "operator.cpp", "device.h")
SCHWARZ_SOURCES = ("schwarz.hip", "schwarz_api.cpp", "schwarz.cpp", "schwarz.h")


def sources_sha(names):
    """First 16 hex digits of the SHA-256 of the named library sources, concatenated in
    the given order."""
    import hashlib
    h = hashlib.sha256()
    for name in names:
        h.update(open(os.path.join(ROOT, "paper_2110_06322_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def apply_sources_sha():
    """Hash of the apply kernel's source and the host code that lays out its tiles and
    work plan."""
    return sources_sha(APPLY_SOURCES)


def measured_traffic(summary="k_apply_pipe_torus_h0.005_counters.md", sources=APPLY_SOURCES):
    """HBM bytes per launch from a committed counter summary, or None when the kernel's
    sources (for the apply also the host code that builds its tiles and work plan)
    changed since the counters were taken."""
    f = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(f):
        return None
    vals = {}
    for line in open(f):
        if ":" in line and line.split(":")[0].strip() in ("traffic_bytes_per_launch", "kernel_source_sha256_16"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != sources_sha(sources) or "traffic_bytes_per_launch" not in vals:
        return None
    return int(vals["traffic_bytes_per_launch"])


def apply_bytes_per_node(d, nA, nG, nrhs=1):
    return 16.0 * nrhs + 8.0 * d * (1.0 + nG / nA)


def timed_applies(op, xs, ys, reps, stream, torch, transpose=False):
    """Mean ms per apply over `reps` rounds of the rotating pairs (events on the stream)."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f = op.apply_T if transpose else op.apply
    e0.record(stream)
    for _ in range(reps):
        for x, y in zip(xs, ys):
            f(x, out=y, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (reps * len(xs))


def rotating(band, torch, dev, inputs, copies=4, seed=10):
    xs = [torch.tensor(inputs.normal(seed + i, 0, band.active_keys), dtype=torch.float64, device=dev)
          for i in range(copies)]
    return xs, [torch.empty_like(xs[0]) for _ in range(copies)]


# ---------------------------------------------------------------- legs
def sphere_leg(cpm, inputs, torch, dev, a, ref):
    """Unit sphere h = 0.02, ORAS 64 boxes: mixed vs FP64 solve to 1e-8 and each solution's
    error against the oracle's reference solution (max-norm, relative), and the same errors
    for untimed solves to the accuracy bars' tolerances (FP64 to 1e-12, mixed to 1e-10)."""
    import numpy as np
    band = cpm.Band("sphere", (1.0,), 3, 0.02, 3)
    op = cpm.Operator(band, 1.0)
    _, cp, _ = band.export()
    nA = band.n_active
    f = torch.tensor(21.0 * inputs.sphere_y4(cp[:nA], 2), dtype=torch.float64, device=dev)
    out = {"workload": "unit sphere h=0.02 p=3 c=1, f=21*Y4 (seed 2), ORAS 64 boxes overlap 2h, local ILU(0)",
           "n_active": nA}
    sols = {}
    for order in (a.ordering, "rcm" if a.ordering == "distance" else "distance"):
        res = {}
        for prec, mode in (("fp32", "mixed"), ("fp64", "fp64")):
            pc = cpm.Precond(op, kind="oras", n_parts=64, overlap=2.0, precision=prec, ordering=order)
            tn = cpm.autotune(op, pc, cache=a.tune_cache)
            times = []
            for _ in range(3):
                u, st = cpm.solve(op, f, pc=pc, rtol=1e-8, mode=mode, max_it=20000)
                times.append(st["ms_total"])
            res[mode] = {"ms": round(float(np.median(times)), 3), "iterations": int(st["iterations"]),
                         "relres": st["relres"], "converged": bool(st["converged"]),
                         "precond_ms": round(tn["precond_ms"], 4)}
            if order == a.ordering:
                sols[mode] = u.cpu().numpy()
                # the accuracy bars: FP64 solved to 1e-12, mixed refined to 1e-10, each against the
                # oracle's reference solution (untimed)
                tight = 1e-12 if mode == "fp64" else 1e-10
                ut, stt = cpm.solve(op, f, pc=pc, rtol=tight, mode=mode, max_it=20000)
                sols[mode + "_tight"] = ut.cpu().numpy()
                res[mode]["tight"] = {"rtol": tight, "iterations": int(stt["iterations"]),
                                      "relres": stt["relres"], "converged": bool(stt["converged"])}
                if mode == "mixed":
                    _, stp = cpm.solve(op, f, pc=pc, rtol=1e-8, mode=mode, max_it=20000, profile=True)
                    res["precond_kernel_ms"] = round(stp["ms_precond"] / max(1, stp["n_precond"]), 5)
                    res["precond_info"] = {"total_nnz": int(pc.info.total_nnz), "total_rows": int(pc.info.total_rows),
                                           "max_levels": int(pc.info.max_levels),
                                           "schwarz_variant": tn["schwarz_variant"]}
        out[order] = res
    # two-level (coarse-first) ORAS of the same partition, and with 512 boxes
    two = {}
    for nb in (64, 512):
        for prec, mode in (("fp32", "mixed"), ("fp64", "fp64")):
            if nb != 64 and mode == "fp64":
                continue
            pc = cpm.Precond(op, kind="oras", n_parts=nb, overlap=2.0, precision=prec, ordering=a.ordering,
                             coarse="first")
            cpm.autotune(op, pc, cache=a.tune_cache)
            times = []
            for _ in range(3):
                u, st = cpm.solve(op, f, pc=pc, rtol=1e-8, mode=mode, max_it=20000)
                times.append(st["ms_total"])
            two[f"{mode}_{nb}_boxes"] = {"ms": round(float(np.median(times)), 3), "iterations": int(st["iterations"]),
                                         "converged": bool(st["converged"])}
            del pc
    out["two_level"] = two
    m = out[a.ordering]
    out["mixed_ms"], out["fp64_ms"] = m["mixed"]["ms"], m["fp64"]["ms"]
    out["speedup_mixed"] = round(m["fp64"]["ms"] / m["mixed"]["ms"], 3)
    out["ordering"] = a.ordering
    if ref is not None:
        rk, rx = ref
        pos = np.searchsorted(rk, band.active_keys)
        ok = bool((rk[pos] == band.active_keys).all())
        if ok:
            sc = float(np.abs(rx).max())
            out["err_vs_oracle_mixed"] = float(np.abs(sols["mixed"] - rx[pos]).max() / sc)
            out["err_vs_oracle_fp64"] = float(np.abs(sols["fp64"] - rx[pos]).max() / sc)
            out["err_vs_oracle_mixed_rtol_1e-10"] = float(np.abs(sols["mixed_tight"] - rx[pos]).max() / sc)
            out["err_vs_oracle_fp64_rtol_1e-12"] = float(np.abs(sols["fp64_tight"] - rx[pos]).max() / sc)
    # the metric kernel on this cache-resident system
    xs, ys = rotating(band, torch, dev, inputs)
    cpm.autotune(op, None)
    timed_applies(op, xs, ys, 2, torch.cuda.current_stream(), torch)
    ms = timed_applies(op, xs, ys, 50, torch.cuda.current_stream(), torch)
    b = apply_bytes_per_node(3, nA, band.n_ghost)
    out["apply"] = {"ms": round(ms, 5), "gnodes_per_s": round(nA / (ms * 1e-3) / 1e9, 3),
                    "hbm_frac": round(b * nA / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "note": "cache-resident: about 16 MB of traffic per apply"}
    return out


def batched_leg(cpm, workloads, torch, ordering):
    """The 48-surface batch to 1e-8 (192 systems, one right-hand side each): mixed precision
    (FP32 factors, FP64 FGMRES-IR) against FP64 (FP64 factors of the same partitions)."""
    import numpy as np
    t0 = time.perf_counter()
    insts = workloads.batched(ordering=ordering)
    t_setup = time.perf_counter() - t0
    print(f"batched: setup {t_setup:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    pcs64 = workloads.preconditioners([i.op for i in insts], [i.meta["n_sub"] for i in insts], "fp64", ordering)
    t_setup64 = time.perf_counter() - t0
    print(f"batched: FP64 preconditioners {t_setup64:.1f} s", file=sys.stderr, flush=True)
    ops1 = [i.op for i in insts for _ in range(4)]
    fs1 = [i.f.view(-1, 4)[:, r].contiguous() for i in insts for r in range(4)]

    def timed(pcs, mode):
        b = cpm.Batch(ops1, pcs, [1] * len(ops1))
        tn = b.autotune()
        b.solve(fs1, rtol=1e-8, mode=mode, max_it=20000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = b.solve(fs1, rtol=1e-8, mode=mode, max_it=20000)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) * 1e3
        del b
        return el, st, tn

    ms1, st1, tune1 = timed([i.pc for i in insts for _ in range(4)], "mixed")
    print(f"batched: mixed {ms1:.0f} ms", file=sys.stderr, flush=True)
    ms64, st64, tune64 = timed([pc for pc in pcs64 for _ in range(4)], "fp64")
    print(f"batched: fp64 {ms64:.0f} ms", file=sys.stderr, flush=True)
    del pcs64
    # the same systems with the two-level (coarse-first) FP32 preconditioners
    t0 = time.perf_counter()
    pcs2 = workloads.preconditioners([i.op for i in insts], [i.meta["n_sub"] for i in insts], "fp32", ordering,
                                     coarse="first")
    t_setup2 = time.perf_counter() - t0
    ms2, st2, _ = timed([pc for pc in pcs2 for _ in range(4)], "mixed")
    print(f"batched: two-level mixed {ms2:.0f} ms", file=sys.stderr, flush=True)
    del pcs2
    its2 = [s["iterations"] for s in st2]
    its1 = [s["iterations"] for s in st1]
    its64 = [s["iterations"] for s in st64]
    return {"workload": "48 surfaces (16 spheres, 16 ellipsoids, 16 tori), h cyclic 0.04/0.02/0.01, p=3, "
                        f"4 N(0,1) RHS each, ORAS 32-512 boxes ({ordering} order), to 1e-8; one right-hand "
                        "side per system",
            "systems": len(st1), "n_active_total": int(sum(i.band.n_active for i in insts)),
            "mixed_ms": round(ms1, 2), "fp64_ms": round(ms64, 2),
            "speedup_mixed": round(ms64 / ms1, 3) if ms1 > 0 else None,
            "iterations_max": int(max(its1)), "iterations_mean": round(float(np.mean(its1)), 1),
            "fp64_iterations_max": int(max(its64)), "fp64_iterations_mean": round(float(np.mean(its64)), 1),
            "max_relres_mixed": float(max(s["relres"] for s in st1)),
            "max_relres_fp64": float(max(s["relres"] for s in st64)),
            "converged": bool(all(s["converged"] for s in st1 + st64)),
            "setup_s": round(t_setup, 2), "fp64_setup_s": round(t_setup64, 2),
            "two_level": {"mixed_ms": round(ms2, 2), "iterations_max": int(max(its2)),
                          "iterations_mean": round(float(np.mean(its2)), 1),
                          "max_relres": float(max(s["relres"] for s in st2)),
                          "converged": bool(all(s["converged"] for s in st2)), "setup_s": round(t_setup2, 2)},
            "tuning": tune1, "tuning_fp64": tune64}


def scaling_leg(cpm, inputs, torch, dev):
    out = []
    band = cpm.Band("torus", (1.0, 0.4), 3, 0.0025, 3)
    op = cpm.Operator(band, 1.0)
    cpm.autotune(op, None)
    xs, ys = rotating(band, torch, dev, inputs)
    timed_applies(op, xs, ys, 1, torch.cuda.current_stream(), torch)
    ms = timed_applies(op, xs, ys, 10, torch.cuda.current_stream(), torch)
    b = apply_bytes_per_node(3, band.n_active, band.n_ghost)
    out.append({"workload": "torus R=1 r=0.4 h=0.0025 p=3 (0.69 GB per apply, 4 rotating pairs)",
                "n_active": band.n_active, "ms": round(ms, 4),
                "gnodes_per_s": round(band.n_active / (ms * 1e-3) / 1e9, 3),
                "hbm_frac": round(b * band.n_active / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "bytes_per_node": round(b, 2)})
    del xs, ys, op, band
    torch.cuda.empty_cache()
    return out


def transpose_leg(cpm, inputs, torch, dev):
    """A^T apply (neighbour sums, then the brick-staged extension transpose) on the adjoint
    workload's torus, h = 0.01."""
    band = cpm.Band("torus", (1.0, 0.4), 3, 0.01, 3)
    op = cpm.Operator(band, 1.0)
    xs, ys = rotating(band, torch, dev, inputs)
    st = torch.cuda.current_stream()
    timed_applies(op, xs, ys, 2, st, torch, transpose=True)
    ms_t = timed_applies(op, xs, ys, 20, st, torch, transpose=True)
    ms_f = timed_applies(op, xs, ys, 20, st, torch)
    nA, nG = band.n_active, band.n_ghost
    # algorithmic bytes per active node of A^T: x (8) and the neighbour sums z over
    # Sigma_A u Sigma_G written and read (2 * 8 (1+g)), closest points (8 d (1+g)),
    # per-brick row lists (about 5.4 entries of 4 B per row, (1+g) rows), output (8)
    g = nG / nA
    b = 8 + 16 * (1 + g) + 24 * (1 + g) + 4 * 5.4 * (1 + g) + 8
    out = {"workload": "torus R=1 r=0.4 h=0.01 p=3 (adjoint system)", "n_active": nA,
           "ms": round(ms_t, 4), "gnodes_per_s": round(nA / (ms_t * 1e-3) / 1e9, 3),
           "hbm_frac": round(b * nA / (ms_t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "bytes_per_node": round(b, 2),
           "forward_ms": round(ms_f, 4)}
    # forward and adjoint solves of the config-4 system: RAS 128 boxes (FP32 factors, of A and
    # of A^T), mixed precision to 1e-8
    import numpy as np
    for name, tr in (("forward_solve", False), ("adjoint_solve", True)):
        pc = cpm.Precond(op, kind="ras", n_parts=128, overlap=2.0, precision="fp32", transpose=tr)
        times = []
        for _ in range(3):
            _, s = cpm.solve(op, xs[0], pc=pc, rtol=1e-8, mode="mixed", max_it=20000, transpose=tr)
            times.append(s["ms_total"])
        out[name] = {"ms": round(float(np.median(times)), 3), "iterations": int(s["iterations"]),
                     "converged": bool(s["converged"])}
        del pc
    return out


def extensions_leg(cpm, inputs, surfaces, torch, dev):
    """Timings of the widened rows: higher-order IMEX steps, the two-level preconditioner's
    iterations, the shifted biharmonic, the fourth-order operator and an open surface."""
    import numpy as np
    out = {}
    st = torch.cuda.current_stream()

    def median_solve(op, f, pc, reps=3, **kw):
        times = []
        for _ in range(reps):
            u, s = cpm.solve(op, f, pc=pc, **kw)
            times.append(s["ms_total"])
        return u, s, float(np.median(times))

    # f1: ARK3(2)4L[2]SA against IMEX Euler, Gray-Scott on the torus h = 0.01, dt = 1
    band = cpm.Band("torus", (1.0, 0.4), 3, 0.01, 3)
    nA = band.n_active
    imex = {"workload": "Gray-Scott torus R=1 r=0.4 h=0.01 p=3, mu=(2e-5,1e-5) F=0.04 k=0.06 dt=1, "
                        "FP32 ORAS 256 boxes, stage solves mixed to 1e-8", "n_active": nA}
    for scheme in ("euler", "ark3"):
        ops = [cpm.Operator(band, cpm.imex_shift(scheme, 1.0, mu)) for mu in (2e-5, 1e-5)]
        pcs = [cpm.Precond(o, kind="oras", n_parts=256, overlap=2.0, precision="fp32") for o in ops]
        im = cpm.Imex(ops, pcs, scheme=scheme, dt=1.0, tune=True)
        g = np.random.default_rng(5)
        ws = [torch.tensor(1.0 - 0.5 * g.random(nA), dtype=torch.float64, device=dev),
              torch.tensor(0.25 * g.random(nA), dtype=torch.float64, device=dev)]
        im.step(ws, nsteps=2, rtol=1e-8, mode="mixed")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = im.step(ws, nsteps=5, rtol=1e-8, mode="mixed")
        torch.cuda.synchronize()
        imex[scheme] = {"ms_per_step": round((time.perf_counter() - t0) * 1e3 / 5, 3),
                        "stage_iterations": [int(x["iterations"]) for x in stats]}
        del im, pcs, ops, ws
    out["imex"] = imex
    del band
    torch.cuda.empty_cache()

    # f2: one level against coarse-first two levels, unit sphere h = 0.01, 256 boxes
    band = cpm.Band("sphere", (1.0,), 3, 0.01, 3)
    op = cpm.Operator(band, 1.0)
    _, cp, _ = band.export()
    f = torch.tensor(21.0 * inputs.sphere_y4(cp[:band.n_active], 2), dtype=torch.float64, device=dev)
    two = {"workload": "unit sphere h=0.01 p=3 c=1, f=21*Y4, FP32 ORAS 256 boxes, mixed to 1e-8",
           "n_active": band.n_active}
    for coarse in ("none", "first"):
        pc = cpm.Precond(op, kind="oras", n_parts=256, overlap=2.0, precision="fp32", coarse=coarse)
        _, s, ms = median_solve(op, f, pc, rtol=1e-8, mode="mixed", max_it=20000)
        two[coarse] = {"iterations": int(s["iterations"]), "ms": round(ms, 3), "converged": bool(s["converged"])}
        del pc
    out["two_level"] = two
    del op, band, f
    torch.cuda.empty_cache()

    # f3: shifted biharmonic (1 + Lap^2) u = f on the unit sphere h = 0.05, and the
    # fourth-order operator with quintic interpolation on the torus h = 0.01
    band = cpm.Band("sphere", (1.0,), 3, 0.05, 3)
    op = cpm.Operator(band, 1.0)
    _, cp, _ = band.export()
    f = torch.tensor(401.0 * inputs.sphere_y4(cp[:band.n_active], 2), dtype=torch.float64, device=dev)
    pc = cpm.Precond(op, kind="oras", n_parts=8, overlap=2.0, precision="fp64", coarse="first")
    _, s, ms = median_solve(op, f, pc, rtol=1e-8, max_it=40000, poly=(1.0, 0.0, 1.0), pc_power=2, restart=60,
                            stagnation_cycles=400)
    _, s2, ms2 = median_solve(op, f, pc, rtol=1e-8, max_it=2000, poly=(1.0, 0.0, 1.0), pc_power=2,
                              pc_inner_rtol=1e-3, pc_inner_max_it=60)
    out["biharmonic"] = {"workload": "(1 + Lap^2) u = 401 Y4, unit sphere h=0.05 p=3, FGMRES to 1e-8, preconditioned "
                                     "by A(1)^-2: two-level ORAS of A(1) applied twice (GMRES(60)), or inner "
                                     "FGMRES solves of A(1) to 1e-3 with that ORAS, twice", "n_active": band.n_active,
                         "squared_oras": {"iterations": int(s["iterations"]), "ms": round(ms, 3),
                                          "converged": bool(s["converged"])},
                         "inner_solves": {"iterations": int(s2["iterations"]), "ms": round(ms2, 3),
                                          "converged": bool(s2["converged"])}}
    del pc, op, band, f
    band = cpm.Band("torus", (1.0, 0.4), 3, 0.01, 5, reach=2)
    op = cpm.Operator(band, 1.0, order=4)
    xs, ys = rotating(band, torch, dev, inputs)
    timed_applies(op, xs, ys, 2, st, torch)
    ms_a = timed_applies(op, xs, ys, 10, st, torch)
    pc = cpm.Precond(op, kind="oras", n_parts=128, overlap=2.0, precision="fp32")
    _, s, ms = median_solve(op, xs[0], pc, rtol=1e-8, mode="mixed", max_it=20000)
    out["fourth_order"] = {"workload": "fourth-order operator, torus R=1 r=0.4 h=0.01 p=5 (reach-2 band), "
                                       "two-kernel apply; solve of a N(0,1) right-hand side, FP32 ORAS 128 boxes "
                                       "(second-order cubic operator), mixed to 1e-8",
                           "n_active": band.n_active, "n_ghost": band.n_ghost, "apply_ms": round(ms_a, 4),
                           "apply_gnodes_per_s": round(band.n_active / (ms_a * 1e-3) / 1e9, 3),
                           "iterations": int(s["iterations"]), "solve_ms": round(ms, 3),
                           "converged": bool(s["converged"])}
    del xs, ys, pc, op, band
    torch.cuda.empty_cache()

    # f4: the hemisphere with the paper's mixed rim (Dirichlet where sin(3 phi) < -0.5)
    fn = surfaces.hemisphere(1.0, lambda phi: np.sin(3.0 * phi) < -0.5)
    t0 = time.perf_counter()
    band = cpm.Band.from_closest_point(fn, 3, 0.01, 3, [-1.6] * 3, [1.6] * 3)
    t_band = time.perf_counter() - t0
    op = cpm.Operator(band, 1.0)
    _, cp, _ = band.export()
    f = torch.tensor(cp[:band.n_active, 2].copy(), dtype=torch.float64, device=dev)
    pc = cpm.Precond(op, kind="oras", n_parts=64, overlap=2.0, precision="fp32")
    _, s, ms = median_solve(op, f, pc, rtol=1e-8, mode="mixed", max_it=20000)
    out["open_surface"] = {"workload": "hemisphere h=0.01 p=3 from a Python closest-point callback, mixed rim, "
                                       "f = z, FP32 ORAS 64 boxes, mixed to 1e-8", "n_active": band.n_active,
                           "band_build_s": round(t_band, 2), "iterations": int(s["iterations"]),
                           "ms": round(ms, 3), "converged": bool(s["converged"])}
    return out


def main():
    a = _args()
    if a.oracle_worker:
        oracle_worker(a.oracle_worker)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported"}))
        sys.exit(2)
    rank0 = int(os.environ.get("RANK", "0")) == 0
    worker = start_oracle() if (rank0 and not a.no_cpu_baseline) else None
    import numpy as np
    import torch

    from paper_2110_06322_amd import _capi, cpm, gray_scott, inputs, surfaces, workloads
    if not os.path.exists(_capi.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    # ---- headline: Gray-Scott on the torus h = 0.005
    t0 = time.perf_counter()
    band = cpm.Band("torus", (1.0, 0.4), 3, 0.005, 3)
    t_band = time.perf_counter() - t0
    t0 = time.perf_counter()
    gs = gray_scott.GrayScott(band, n_parts=1024, mode="mixed", precision="fp32", rtol=1e-8, tune=True,
                              tune_cache=a.tune_cache, ordering=a.gs_ordering)
    t_gs = time.perf_counter() - t0
    print(f"gray-scott: band {t_band:.1f} s, setup {t_gs:.1f} s", file=sys.stderr, flush=True)
    op = gs.ops[0]
    nA, nG = band.n_active, band.n_ghost
    xs, ys = rotating(band, torch, dev, inputs)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]

    def step(k=None):
        st = gs.step()
        if k is not None:
            ev[k][0].record(stream)
        for r in range(a.apply_burst):
            op.apply(xs[r % 4], out=ys[r % 4], stream=stream)
        if k is not None:
            ev[k][1].record(stream)
        return st

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    # ---- timed region: K steps
    t_start = time.perf_counter()
    stats = [step(k) for k in range(a.steps)]
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_step = t_total * 1e3 / a.steps
    ms_apply = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev])) / a.apply_burst
    print(f"gray-scott: {ms_step:.2f} ms per step, apply {ms_apply * 1e3:.1f} us", file=sys.stderr, flush=True)
    # Gray-Scott step time alone, mixed (from the current state), then FP64 factors + FP64 GMRES
    def gs_steps(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = []
        for _ in range(n):
            st = gs.step()
            its.append(max(s["iterations"] for s in st))
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n, its

    gs_mixed_ms, its_m = gs_steps(5)
    state = (gs.u.clone(), gs.v.clone())
    t0 = time.perf_counter()
    pcs64 = workloads.preconditioners(gs.ops, [1024, 1024], "fp64", a.gs_ordering)
    t_pc64 = time.perf_counter() - t0
    gs64 = gray_scott.GrayScott(band, n_parts=0, mode="fp64", rtol=1e-8, ops=gs.ops, pcs=pcs64, tune=True,
                                tune_cache=a.tune_cache)
    gs64.u.copy_(state[0])
    gs64.v.copy_(state[1])
    gs64.step()   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its_64 = []
    for _ in range(5):
        st = gs64.step()
        its_64.append(max(s["iterations"] for s in st))
    torch.cuda.synchronize()
    gs_fp64_ms = (time.perf_counter() - t0) * 1e3 / 5
    u = gs.u
    gray = {"workload": "Gray-Scott torus R=1 r=0.4 h=0.005 p=3, mu=(2e-5,1e-5) F=0.04 k=0.06 dt=1, ORAS 1024 "
                        f"boxes ({a.gs_ordering} order), to 1e-8, warm starts",
            "n_active": nA, "mixed_step_ms": round(gs_mixed_ms, 3), "fp64_step_ms": round(gs_fp64_ms, 3),
            "speedup_mixed": round(gs_fp64_ms / gs_mixed_ms, 3), "iterations_max_mixed": int(max(its_m)),
            "iterations_max_fp64": int(max(its_64)), "setup_s": round(t_band + t_gs, 2),
            "fp64_setup_s": round(t_pc64, 2), "u_min": float(u.min()), "u_max": float(u.max()),
            "finite": bool(torch.isfinite(u).all()), "tuning": gs.tuning}
    del gs64, pcs64
    torch.cuda.empty_cache()

    gnodes = nA / (ms_apply * 1e-3) / 1e9
    b_alg = apply_bytes_per_node(3, nA, nG)
    achieved = b_alg * nA / (ms_apply * 1e-3) / 1e9
    apply_kernel = "k_apply_pipe<3,3>" if (gs.tuning or {}).get("apply_variant", 0) == 0 else "k_apply_tile<3,3,1>"

    legs = {}
    legs["apply_scaling"] = None if a.no_scaling else scaling_leg(cpm, inputs, torch, dev)
    legs["apply_T"] = None if a.no_scaling else transpose_leg(cpm, inputs, torch, dev)
    legs["batched"] = None if a.no_batched else batched_leg(cpm, workloads, torch, a.batched_ordering)
    oracle = finish_oracle(*worker) if worker is not None else {}
    legs["solve"] = sphere_leg(cpm, inputs, torch, dev, a, oracle.get("ref"))
    legs["extensions"] = None if a.no_extensions else extensions_leg(cpm, inputs, surfaces, torch, dev)

    out = {
        "metric": METRIC,
        "value": round(gnodes, 3),
        "unit": "Gnodes/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Gray-Scott on the torus R=1 r=0.4, h=0.005 on [-2,2]^3, p=3: per step two batched "
                               "shifted solves (FP32 ORAS 1024 boxes, FP64 FGMRES-IR to 1e-8) and a burst of "
                               f"{a.apply_burst} operator applies over 4 rotating vector pairs",
                   "n_active": nA, "n_ghost": nG, "n_band": band.n_band},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": apply_kernel, "bytes_per_node": round(b_alg, 2),
                     "units_per_launch": nA},
        "gray_scott": gray,
        **legs,
    }
    if oracle.get("cpu.json"):
        cb = oracle["cpu.json"]
        if oracle.get("ref.json"):
            cb["reference_solve"] = oracle["ref.json"]
        out["cpu_baseline"] = cb
    print(json.dumps(out))


if __name__ == "__main__":
    main()
