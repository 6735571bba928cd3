"""Semi-implicit Gray-Scott reaction-diffusion on a surface (paper Sec. 4.1.5,
eq. grayscott, with the IMEX splitting of Sec. 1): the reaction is advanced
explicitly, the diffusion implicitly by shifted CPM solves of both species
that run together as one batch, each warm-started, with FP32 Schwarz
preconditioners inside FP64 FGMRES.

scheme "euler": IMEX Euler, one solve per species and step (c_w = 1/(mu_w dt));
scheme "ark3": the library's ARK3(2)4L[2]SA integrator (cpm.Imex), three
stage solves per species and step at c_w = 1/(dt gamma mu_w).

State can be saved and restored (`checkpoint` / `resume`) as .npz files.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import cpm, inputs
from ._capi import check, lib


class GrayScott:
    def __init__(self, band: cpm.Band, mu=(2e-5, 1e-5), F=0.04, k=0.06, dt=1.0, n_parts=1024,
                 kind="oras", precision="fp32", mode="mixed", rtol=1e-8, seed=5, device="cuda", tune=False,
                 tune_cache=None, ordering="rcm", ops=None, pcs=None, scheme="euler"):
        """ops / pcs: existing operators (at the scheme's stage shifts) and preconditioners to share, e.g.
        to run the same system with factors of another precision; otherwise they are built
        here (n_parts = 0: no preconditioner)."""
        self.band, self.mu, self.F, self.k, self.dt = band, tuple(mu), F, k, dt
        self.rtol, self.mode, self.scheme = rtol, mode, scheme
        shifts = [cpm.imex_shift(scheme, dt, m) for m in self.mu]
        self.ops = list(ops) if ops is not None else [cpm.Operator(band, c) for c in shifts]
        for op, c in zip(self.ops, shifts):
            if abs(op.c - c) > 1e-12 * c:
                raise ValueError("operator shift does not match the scheme's stage shift")
        if pcs is not None:
            self.pcs = list(pcs)
        elif n_parts > 0:
            from .workloads import preconditioners
            self.pcs = preconditioners(self.ops, [n_parts] * len(self.ops), precision, ordering, kind=kind)
        else:
            self.pcs = [None, None]
        self.batch, self.tuning, self.imex = None, None, None
        if scheme == "euler":
            self.batch = cpm.Batch(self.ops, self.pcs, [1, 1])
            self.tuning = self.batch.autotune(cache=tune_cache) if tune else None
        else:
            self.imex = cpm.Imex(self.ops, self.pcs, scheme=scheme, kind="gray_scott", dt=dt, mu=self.mu, F=F, k=k,
                                 tune=tune)
        u0, v0 = inputs.gray_scott_ic(band.active_keys, seed)
        self.u = torch.tensor(u0, dtype=torch.float64, device=device)
        self.v = torch.tensor(v0, dtype=torch.float64, device=device)
        self.fu, self.fv = torch.empty_like(self.u), torch.empty_like(self.v)
        self.step_count = 0
        self.seed = seed
        self.last_stats = None

    def rhs(self, stream=None):
        s = torch.cuda.current_stream() if stream is None else stream
        check(lib().cpm_gray_scott_rhs(self.u.numel(), C.c_void_p(self.u.data_ptr()), C.c_void_p(self.v.data_ptr()),
                                       self.F, self.k, self.dt, self.mu[0], self.mu[1],
                                       C.c_void_p(self.fu.data_ptr()), C.c_void_p(self.fv.data_ptr()),
                                       C.c_void_p(s.cuda_stream)))

    def step(self):
        if self.imex is not None:
            stats = self.imex.step([self.u, self.v], t=self.step_count * self.dt, nsteps=1, rtol=self.rtol,
                                   mode=self.mode, max_it=20000)
            if not all(s["converged"] for s in stats):
                raise RuntimeError(f"Gray-Scott step {self.step_count} did not converge: {stats}")
            self.step_count += 1
            self.last_stats = stats
            return stats
        self.rhs()
        # warm start: the solves begin from the current state
        us, stats = self.batch.solve([self.fu, self.fv], [self.u, self.v], rtol=self.rtol, mode=self.mode,
                                     max_it=20000)
        if not all(s["converged"] for s in stats):
            raise RuntimeError(f"Gray-Scott step {self.step_count} did not converge: {stats}")
        self.step_count += 1
        self.last_stats = stats
        return stats

    def checkpoint(self, path):
        np.savez(path, step=self.step_count, u=self.u.cpu().numpy(), v=self.v.cpu().numpy(), seed=self.seed,
                 mu=np.array(self.mu), F=self.F, k=self.k, dt=self.dt)

    def resume(self, path):
        z = np.load(path)
        if z["u"].shape[0] != self.u.numel():
            raise ValueError("checkpoint belongs to another band")
        self.u.copy_(torch.from_numpy(z["u"]))
        self.v.copy_(torch.from_numpy(z["v"]))
        self.step_count = int(z["step"])
