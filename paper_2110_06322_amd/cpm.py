"""Python binding of the CPM library: thin wrappers that marshal torch/numpy
arguments into the C ABI (include/cpm.h). Every step of the hot path runs in
the library's HIP kernels; torch only provides device memory and streams.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _capi
from ._capi import check, lib

SURFACES = {"circle": 0, "sphere": 1, "torus": 2, "ellipsoid": 3}
PC_KIND = {"none": 0, "ras": 1, "oras": 2}
SUBSOLVER = {"ilu0": 0, "lu": 1}
PRECISION = {"fp64": 0, "fp32": 1}
MODE = {"fp64": 0, "mixed": 1}
ORDERING = {"rcm": 0, "distance": 1}


def _torch():
    return torch


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    if not t.is_cuda or t.dtype != _torch().float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def device_count() -> int:
    return int(lib().cpm_device_count())


class Band:
    """The CPM band (Sigma_A, Sigma_G) of an analytic surface, built on the host."""

    def __init__(self, kind: str, params, d: int, h: float, p: int, lo=None, hi=None,
                 gamma: float = 0.0, center=(0.0, 0.0, 0.0)):
        s = _capi.Surface()
        s.kind = SURFACES[kind]
        for k, v in enumerate(params):
            s.params[k] = float(v)
        for k, v in enumerate(center):
            s.center[k] = float(v)
        lo = [-2.0] * d if lo is None else list(lo)
        hi = [2.0] * d if hi is None else list(hi)
        arr = C.c_double * d
        h_ = C.c_void_p()
        check(lib().cpm_band_build(C.byref(s), d, float(h), p, arr(*lo), arr(*hi), float(gamma), C.byref(h_)))
        self._h = h_
        self.kind, self.params, self.d, self.h, self.p = kind, tuple(params), d, h, p
        info = _capi.BandInfo()
        check(lib().cpm_band_get_info(self._h, C.byref(info)))
        self.info = info
        self.n_active = int(info.n_active)
        self.n_ghost = int(info.n_ghost)
        self.n_band = int(info.n_band)
        self.gamma = float(info.gamma)
        self.shape = tuple(int(info.shape[k]) for k in range(d))
        self.lo = np.array([info.lo[k] for k in range(d)])
        self._export = None

    def export(self):
        """(gidx [n, d] int32, cp [n, d] float64, kind [n] uint8), Sigma_A first."""
        if self._export is None:
            n = self.n_active + self.n_ghost
            g = np.zeros((n, self.d), dtype=np.int32)
            cp = np.zeros((n, self.d), dtype=np.float64)
            kd = np.zeros(n, dtype=np.uint8)
            check(lib().cpm_band_export(self._h, g.ctypes.data_as(C.c_void_p), cp.ctypes.data_as(C.c_void_p),
                                        kd.ctypes.data_as(C.c_void_p)))
            self._export = (g, cp, kd)
        return self._export

    @property
    def active_keys(self):
        g, _, _ = self.export()
        key = np.zeros(self.n_active, dtype=np.int64)
        for k in range(self.d):
            key = key * self.shape[k] + g[:self.n_active, k].astype(np.int64)
        return key

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None and self._h.value:
                lib().cpm_band_destroy(self._h)
        except Exception:
            pass


class Operator:
    """A = (c + 2d/h^2) I - h^-2 O E on a band, resident on the GPU."""

    def __init__(self, band: Band, c: float, stream=None):
        h_ = C.c_void_p()
        check(lib().cpm_operator_create(band._h, float(c), _stream(stream), C.byref(h_)))
        self._h = h_
        self.band = band
        self.n_active = band.n_active
        self.d, self.p, self.h = band.d, band.p, band.h

    @property
    def c(self) -> float:
        return float(lib().cpm_operator_get_shift(self._h))

    def set_shift(self, c: float):
        check(lib().cpm_operator_set_shift(self._h, float(c)))

    def _out(self, x, nrhs, out):
        torch = _torch()
        return torch.empty_like(x) if out is None else out

    def apply(self, x, out=None, nrhs: int = 1, stream=None):
        y = self._out(x, nrhs, out)
        check(lib().cpm_apply(self._h, _dptr(x), _dptr(y), nrhs, _stream(stream)))
        return y

    def apply_T(self, x, out=None, nrhs: int = 1, stream=None):
        y = self._out(x, nrhs, out)
        check(lib().cpm_apply_T(self._h, _dptr(x), _dptr(y), nrhs, _stream(stream)))
        return y

    def extend(self, u, out=None, stream=None):
        torch = _torch()
        n = self.band.n_active + self.band.n_ghost
        v = torch.empty(n, dtype=torch.float64, device=u.device) if out is None else out
        check(lib().cpm_extend_apply(self._h, _dptr(u), _dptr(v), _stream(stream)))
        return v

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None and self._h.value:
                lib().cpm_operator_destroy(self._h)
        except Exception:
            pass


@dataclass
class PrecondOptions:
    kind: str = "oras"
    n_parts: int = 64
    overlap: float = 2.0
    alpha: float = 4.0
    alpha_cross: float = 20.0
    subsolver: str = "ilu0"
    precision: str = "fp64"
    transpose: bool = False
    ordering: str = "rcm"

    def to_c(self):
        o = _capi.PrecondOpts()
        o.kind = PC_KIND[self.kind]
        o.n_parts = int(self.n_parts)
        o.overlap = float(self.overlap)
        o.alpha = float(self.alpha)
        o.alpha_cross = float(self.alpha_cross)
        o.subsolver = SUBSOLVER[self.subsolver]
        o.precision = PRECISION[self.precision]
        o.transpose = int(bool(self.transpose))
        o.ordering = ORDERING[self.ordering]
        return o


class Precond:
    """(O)RAS preconditioner with ILU(0) (or exact LU) local solves."""

    def __init__(self, op: Operator, opts: PrecondOptions | None = None, **kw):
        opts = opts or PrecondOptions(**kw)
        h_ = C.c_void_p()
        co = opts.to_c()
        check(lib().cpm_precond_create(op._h, C.byref(co), C.byref(h_)))
        self._h = h_
        self.op = op
        self.opts = opts
        info = _capi.PrecondInfo()
        check(lib().cpm_precond_get_info(self._h, C.byref(info)))
        self.info = info

    def export_partition(self):
        n = self.op.n_active
        owner = np.zeros(n, dtype=np.int32)
        ptr = np.zeros(self.info.n_parts + 1, dtype=np.int64)
        idx = np.zeros(self.info.total_rows, dtype=np.int32)
        check(lib().cpm_precond_export_partition(self._h, owner.ctypes.data_as(C.c_void_p),
                                                  ptr.ctypes.data_as(C.c_void_p), idx.ctypes.data_as(C.c_void_p)))
        return owner, ptr, idx

    def apply(self, r, out=None, nrhs: int = 1, stream=None):
        torch = _torch()
        z = torch.empty_like(r) if out is None else out
        check(lib().cpm_precond_apply(self._h, _dptr(r), _dptr(z), nrhs, _stream(stream)))
        return z

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None and self._h.value:
                lib().cpm_precond_destroy(self._h)
        except Exception:
            pass


def autotune(op: Operator, pc: Precond | None = None, nrhs: int = 1, cache: str | None = None,
             force: bool = False, stream=None) -> dict:
    """Pick the fastest apply / subdomain-solve kernels for this operator (and
    preconditioner); choices are cached per shape class in the JSON file `cache`."""
    r = _capi.TuneResult()
    path = None if cache is None else str(cache).encode()
    check(lib().cpm_autotune(op._h, None if pc is None else pc._h, int(nrhs), path, int(bool(force)),
                             _stream(stream), C.byref(r)))
    return {f: getattr(r, f) for f, _ in _capi.TuneResult._fields_}


@dataclass
class SolveOptions:
    restart: int = 30
    rtol: float = 1e-10
    atol: float = 0.0
    max_it: int = 10000
    mode: str = "fp64"
    transpose: bool = False
    use_graph: bool = False
    inner_rtol: float = 1e-4
    stagnation_cycles: int = 50
    profile: bool = False

    def to_c(self):
        o = _capi.SolveOpts()
        o.restart = int(self.restart)
        o.rtol = float(self.rtol)
        o.atol = float(self.atol)
        o.max_it = int(self.max_it)
        o.mode = MODE[self.mode]
        o.transpose = int(bool(self.transpose))
        o.use_graph = int(bool(self.use_graph))
        o.inner_rtol = float(self.inner_rtol)
        o.stagnation_cycles = int(self.stagnation_cycles)
        o.profile = int(bool(self.profile))
        return o


def _stats_dict(s):
    return {f: getattr(s, f) for f, _ in _capi.SolveStats._fields_}


def solve(op: Operator, f, pc: Precond | None = None, u=None, nrhs: int = 1, opts: SolveOptions | None = None,
          stream=None, raise_on_fail: bool = False, **kw):
    """Solve A u = f (or A^T u = f) with restarted FGMRES on the GPU; returns (u, stats)."""
    torch = _torch()
    opts = opts or SolveOptions(**kw)
    u = torch.zeros_like(f) if u is None else u
    st = _capi.SolveStats()
    co = opts.to_c()
    code = lib().cpm_solve(op._h, pc._h if pc is not None else None, _dptr(f), _dptr(u), nrhs,
                           C.byref(co), C.byref(st), _stream(stream))
    if code not in (_capi.CPM_OK, 6) or (raise_on_fail and code != _capi.CPM_OK):
        check(code)
    return u, _stats_dict(st)


class Batch:
    """Many operators / preconditioners / right-hand sides advanced in shared launches."""

    def __init__(self, ops, pcs=None, nrhs=None):
        n = len(ops)
        pcs = pcs or [None] * n
        nrhs = nrhs or [1] * n
        self._ops, self._pcs = list(ops), list(pcs)
        self.nrhs = list(nrhs)
        oa = (C.c_void_p * n)(*[o._h.value for o in ops])
        pa = (C.c_void_p * n)(*[(p._h.value if p is not None else None) for p in pcs])
        ra = (C.c_int32 * n)(*nrhs)
        h_ = C.c_void_p()
        check(lib().cpm_batch_create(n, oa, pa, ra, C.byref(h_)))
        self._h = h_

    def solve(self, fs, us=None, opts: SolveOptions | None = None, stream=None, **kw):
        torch = _torch()
        opts = opts or SolveOptions(**kw)
        us = us or [torch.zeros_like(f) for f in fs]
        n = len(fs)
        fa = (C.c_void_p * n)(*[f.data_ptr() for f in fs])
        ua = (C.c_void_p * n)(*[u.data_ptr() for u in us])
        nsys = sum(self.nrhs)
        st = (_capi.SolveStats * nsys)()
        co = opts.to_c()
        code = lib().cpm_batch_solve(self._h, fa, ua, C.byref(co), st, _stream(stream))
        if code not in (_capi.CPM_OK, 6):
            check(code)
        return us, [_stats_dict(s) for s in st]

    def autotune(self, cache: str | None = None, force: bool = False, stream=None) -> dict:
        """Pick the batch's apply and subdomain-solve kernels by timing them on the whole batch."""
        r = _capi.TuneResult()
        path = None if cache is None else str(cache).encode()
        check(lib().cpm_batch_autotune(self._h, path, int(bool(force)), _stream(stream), C.byref(r)))
        return {f: getattr(r, f) for f, _ in _capi.TuneResult._fields_}

    def apply(self, xs, ys=None, stream=None):
        torch = _torch()
        ys = ys or [torch.empty_like(x) for x in xs]
        n = len(xs)
        xa = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        ya = (C.c_void_p * n)(*[y.data_ptr() for y in ys])
        check(lib().cpm_batch_apply(self._h, xa, ya, _stream(stream)))
        return ys

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None and self._h.value:
                lib().cpm_batch_destroy(self._h)
        except Exception:
            pass


class CPMSolve(torch.autograd.Function):
    """u = A(c)^-1 f as a differentiable function of (f, c).

    A(c) = c I + K with K independent of c, so for a loss L(u) with
    g = dL/du: A^T lambda = g, dL/df = lambda, dL/dc = -lambda . u.
    Forward and backward both run GPU FGMRES; the backward solve uses A^T and
    a preconditioner built on A^T when one is given. Call as
    CPMSolve.apply(f, c, op, pc, pc_T, opts, adjoint_rtol) with c a 0-d tensor;
    adjoint_rtol (default opts.rtol) sets the A^T solve's tolerance, since the
    attainable residual of either solve is about eps |A| |u| / |f|.
    """

    @staticmethod
    def forward(ctx, f, c, op, pc=None, pc_T=None, opts=None, adjoint_rtol=None):
        opts = opts or SolveOptions(rtol=1e-12)
        cval = float(c)
        if op.c != cval:
            op.set_shift(cval)
        u, st = solve(op, f.detach().contiguous(), pc=pc, opts=opts)
        if not st["converged"]:
            raise RuntimeError(f"forward solve did not converge: {st}")
        ctx.save_for_backward(u)
        ctx.op, ctx.pc_T, ctx.opts = op, pc_T, opts
        ctx.adjoint_rtol = opts.rtol if adjoint_rtol is None else float(adjoint_rtol)
        ctx.c_meta = (c.device, c.dtype) if torch.is_tensor(c) else (u.device, u.dtype)
        return u

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        o = ctx.opts
        ot = SolveOptions(restart=o.restart, rtol=ctx.adjoint_rtol, atol=o.atol, max_it=o.max_it, mode="fp64",
                          transpose=True, stagnation_cycles=o.stagnation_cycles)
        lam, st = solve(ctx.op, g.contiguous(), pc=ctx.pc_T, opts=ot)
        if not st["converged"]:
            raise RuntimeError(f"adjoint solve did not converge: {st}")
        gc = -torch.dot(lam, u)
        return lam, gc.reshape(()).to(device=ctx.c_meta[0], dtype=ctx.c_meta[1]), None, None, None, None, None
