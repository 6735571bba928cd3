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
COARSE = {"none": 0, "additive": 1, "first": 2}


def _torch():
    return torch


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def check_vec(t, n: int, what: str = "vector", on_device: bool = False):
    """Validate a vector before its address goes to the library: a torch tensor,
    float64, contiguous, exactly n elements and (on_device, checked when the
    address is taken, after every argument's size) on a CUDA (HIP) device.
    Raises TypeError / ValueError; nothing is passed on when a check fails."""
    torch = _torch()
    if not torch.is_tensor(t):
        raise TypeError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != torch.float64:
        raise ValueError(f"{what}: expected float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{what}: expected {n} elements, got {t.numel()}")
    if on_device and not t.is_cuda:
        raise ValueError(f"{what}: must be a CUDA (HIP) device tensor")
    return t


def check_nrhs(nrhs: int):
    if nrhs not in (1, 2, 4):
        raise ValueError(f"nrhs must be 1, 2 or 4, got {nrhs}")
    return int(nrhs)


def check_disjoint(a, b, what: str):
    """The library's outputs must not overlap its inputs."""
    a0, b0 = a.data_ptr(), b.data_ptr()
    if a.numel() and b.numel() and a0 < b0 + b.numel() * b.element_size() and b0 < a0 + a.numel() * a.element_size():
        raise ValueError(f"{what} must not overlap")


def check_count(seq, n: int, what: str):
    if len(seq) != n:
        raise ValueError(f"{what}: expected {n} entries (one per instance), got {len(seq)}")
    return list(seq)


def _dptr(t, n: int, what: str = "vector"):
    return C.c_void_p(check_vec(t, n, what, on_device=True).data_ptr())


def device_count() -> int:
    return int(lib().cpm_device_count())


class Band:
    """The CPM band (Sigma_A, Sigma_G) of an analytic surface, built on the host."""

    def __init__(self, kind: str, params, d: int, h: float, p: int, lo=None, hi=None,
                 gamma: float = 0.0, center=(0.0, 0.0, 0.0), reach: int = 1):
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
        if reach == 1:
            check(lib().cpm_band_build(C.byref(s), d, float(h), p, arr(*lo), arr(*hi), float(gamma), C.byref(h_)))
        else:
            check(lib().cpm_band_build_reach(C.byref(s), _capi.CP_CALLBACK(), None, d, float(h), p, arr(*lo),
                                             arr(*hi), float(gamma), int(reach), C.byref(h_)))
        self._h = h_
        self._init_info(kind, params, d, h, p)

    @classmethod
    def from_closest_point(cls, fn, d: int, h: float, p: int, lo, hi, gamma: float = 0.0, name: str = "user",
                           reach: int = 1):
        """Band of a surface given by a closest point function (cpm_band_build_user).

        fn(x) with x an (n, d) float64 array returns (cp, flag): the (n, d) closest points
        and an (n,) integer array, 1 where the closest point lies on a boundary part with
        homogeneous Dirichlet conditions (those rows are mirrored), else 0. The function
        only evaluates the surface; the band is built by the library."""
        err = []

        def cb(n, xp, cpp, flp, ctx):
            try:
                x = np.ctypeslib.as_array(xp, shape=(n, d))
                cp, flag = fn(np.array(x))
                np.ctypeslib.as_array(cpp, shape=(n, d))[:] = np.asarray(cp, dtype=np.float64).reshape(n, d)
                np.ctypeslib.as_array(flp, shape=(n,))[:] = np.asarray(flag, dtype=np.int32).reshape(n)
                return 0
            except Exception as e:  # reported after the call returns
                err.append(e)
                return 1
        self = cls.__new__(cls)
        c_cb = _capi.CP_CALLBACK(cb)
        arr = C.c_double * d
        lo = list(lo)
        hi = list(hi)
        h_ = C.c_void_p()
        if reach == 1:
            code = lib().cpm_band_build_user(c_cb, None, d, float(h), p, arr(*lo), arr(*hi), float(gamma),
                                             C.byref(h_))
        else:
            code = lib().cpm_band_build_reach(None, c_cb, None, d, float(h), p, arr(*lo), arr(*hi), float(gamma),
                                              int(reach), C.byref(h_))
        if err:
            raise err[0]
        check(code)
        self._h = h_
        self._init_info(name, (), d, h, p)
        return self

    def _init_info(self, kind, params, d, h, p):
        self.kind, self.params, self.d, self.h, self.p = kind, tuple(params), d, h, p
        info = _capi.BandInfo()
        check(lib().cpm_band_get_info(self._h, C.byref(info)))
        self.info = info
        self.n_active = int(info.n_active)
        self.n_ghost = int(info.n_ghost)
        self.n_band = int(info.n_band)
        self.gamma = float(info.gamma)
        self.reach = int(info.reach)
        self.shape = tuple(int(info.shape[k]) for k in range(d))
        self.lo = np.array([info.lo[k] for k in range(d)])
        self._export = None

    def export_interp(self):
        """(ip [n, d], sign [n]): interpolation point and sign of every extension row."""
        n = self.n_active + self.n_ghost
        ip = np.zeros((n, self.d), dtype=np.float64)
        sg = np.zeros(n, dtype=np.float64)
        check(lib().cpm_band_export_interp(self._h, ip.ctypes.data_as(C.c_void_p), sg.ctypes.data_as(C.c_void_p)))
        return ip, sg

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
    """A = (c + 2d/h^2) I - h^-2 O E on a band, resident on the GPU (order 4: the
    fourth-order stencil, on a band of reach 2; lds_bytes: LDS budget per tile of the
    fused apply, 0 for the default 64 KiB)."""

    def __init__(self, band: Band, c: float, stream=None, order: int = 2, lds_bytes: int = 0):
        h_ = C.c_void_p()
        if order == 2 and lds_bytes == 0:
            check(lib().cpm_operator_create(band._h, float(c), _stream(stream), C.byref(h_)))
        else:
            o = _capi.OperatorOpts()
            check(lib().cpm_operator_opts_default(C.byref(o)))
            o.order = int(order)
            o.apply_lds_bytes = int(lds_bytes)
            check(lib().cpm_operator_create_ex(band._h, float(c), C.byref(o), _stream(stream), C.byref(h_)))
        self.order = order
        self._h = h_
        self.band = band
        self.n_active = band.n_active
        self.d, self.p, self.h = band.d, band.p, band.h

    @property
    def info(self) -> dict:
        i = _capi.OperatorInfo()
        check(lib().cpm_operator_get_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in _capi.OperatorInfo._fields_}

    @property
    def c(self) -> float:
        return float(lib().cpm_operator_get_shift(self._h))

    def set_shift(self, c: float):
        check(lib().cpm_operator_set_shift(self._h, float(c)))

    def _io(self, x, out, nrhs):
        torch = _torch()
        n = self.n_active * check_nrhs(nrhs)
        check_vec(x, n, "x")
        y = torch.empty_like(x) if out is None else check_vec(out, n, "out")
        check_disjoint(x, y, "x and out")
        return x, y, n

    def apply(self, x, out=None, nrhs: int = 1, stream=None):
        x, y, n = self._io(x, out, nrhs)
        check(lib().cpm_apply(self._h, _dptr(x, n), _dptr(y, n), nrhs, _stream(stream)))
        return y

    def poly_apply(self, coef, x, out=None, nrhs: int = 1, stream=None):
        """y = sum_k coef[k] L^k x with L = c I - A(c), the band's Laplace-Beltrami operator
        (1 to 5 coefficients)."""
        coef = [float(a) for a in coef]
        if not 1 <= len(coef) <= 5:
            raise ValueError("1 to 5 polynomial coefficients")
        x, y, n = self._io(x, out, nrhs)
        ca = (C.c_double * len(coef))(*coef)
        check(lib().cpm_poly_apply(self._h, len(coef), ca, _dptr(x, n), _dptr(y, n), nrhs, _stream(stream)))
        return y

    def apply_T(self, x, out=None, nrhs: int = 1, stream=None):
        x, y, n = self._io(x, out, nrhs)
        check(lib().cpm_apply_T(self._h, _dptr(x, n), _dptr(y, n), nrhs, _stream(stream)))
        return y

    def apply_T_noalloc(self, x, out, nrhs: int = 1, stream=None):
        """y = A^T x through the allocation-free entry point (its intermediate sums live in
        a static device array shared by every call on the GPU); `out` must be given."""
        x, y, n = self._io(x, out, nrhs)
        check(lib().cpm_apply_T_noalloc(self._h, _dptr(x, n), _dptr(y, n), nrhs, _stream(stream)))
        return y

    def extend(self, u, out=None, stream=None):
        torch = _torch()
        n = self.band.n_active + self.band.n_ghost
        check_vec(u, self.n_active, "u")
        v = torch.empty(n, dtype=torch.float64, device=u.device) if out is None else check_vec(out, n, "out")
        check_disjoint(u, v, "u and out")
        check(lib().cpm_extend_apply(self._h, _dptr(u, self.n_active), _dptr(v, n), _stream(stream)))
        return v

    def shift_gradient(self, lam, u, nrhs: int = 1, out=None, stream=None):
        """dL/dc = -lambda . u as a one-element device tensor (reduced by the library in a
        fixed order), for u = A(c)^-1 f and the adjoint solution lambda."""
        torch = _torch()
        n = self.n_active * check_nrhs(nrhs)
        check_vec(lam, n, "lambda")
        check_vec(u, n, "u")
        g = torch.empty(1, dtype=torch.float64, device=u.device) if out is None else check_vec(out, 1, "out")
        check_disjoint(lam, g, "lambda and out")
        check_disjoint(u, g, "u and out")
        check(lib().cpm_shift_gradient(self._h, _dptr(lam, n), _dptr(u, n), nrhs, _dptr(g, 1), _stream(stream)))
        return g

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
    coarse: str = "none"

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
        o.coarse = COARSE[self.coarse]
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
        n = self.op.n_active * check_nrhs(nrhs)
        check_vec(r, n, "r")
        z = torch.empty_like(r) if out is None else check_vec(out, n, "out")
        check_disjoint(r, z, "r and out")
        check(lib().cpm_precond_apply(self._h, _dptr(r, n), _dptr(z, n), nrhs, _stream(stream)))
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
    # operator algebra: solve P(L) u = f with P(L) = sum_k poly[k] L^k (empty: A u = f)
    poly: tuple = ()
    # preconditioner applications per step (2 with the (O)RAS of A(sqrt(c0)) for c0 + L^2)
    pc_power: int = 1
    # > 0: each preconditioner application is an inner FGMRES solve of A w = v to this
    # relative tolerance (at most pc_inner_max_it steps), preconditioned by the (O)RAS
    pc_inner_rtol: float = 0.0
    pc_inner_max_it: int = 30

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
        coef = [float(a) for a in self.poly]
        if len(coef) > 5:
            raise ValueError("at most 5 polynomial coefficients (degree 4)")
        o.poly_n = len(coef)
        for k, a in enumerate(coef):
            o.poly_coef[k] = a
        o.pc_power = int(self.pc_power)
        o.pc_inner_rtol = float(self.pc_inner_rtol)
        o.pc_inner_max_it = int(self.pc_inner_max_it)
        return o


def _stats_dict(s):
    return {f: getattr(s, f) for f, _ in _capi.SolveStats._fields_}


def solve(op: Operator, f, pc: Precond | None = None, u=None, nrhs: int = 1, opts: SolveOptions | None = None,
          stream=None, raise_on_fail: bool = False, **kw):
    """Solve A u = f (or A^T u = f) with restarted FGMRES on the GPU; returns (u, stats)."""
    torch = _torch()
    opts = opts or SolveOptions(**kw)
    n = op.n_active * check_nrhs(nrhs)
    check_vec(f, n, "f")
    u = torch.zeros_like(f) if u is None else check_vec(u, n, "u")
    check_disjoint(f, u, "f and u")
    if pc is not None and pc.op is not op:
        raise ValueError("the preconditioner was built for another operator")
    st = _capi.SolveStats()
    co = opts.to_c()
    code = lib().cpm_solve(op._h, pc._h if pc is not None else None, _dptr(f, n), _dptr(u, n), nrhs,
                           C.byref(co), C.byref(st), _stream(stream))
    if code not in (_capi.CPM_OK, 6) or (raise_on_fail and code != _capi.CPM_OK):
        check(code)
    return u, _stats_dict(st)


class Batch:
    """Many operators / preconditioners / right-hand sides advanced in shared launches."""

    def __init__(self, ops, pcs=None, nrhs=None):
        n = len(ops)
        pcs = check_count(pcs or [None] * n, n, "pcs")
        nrhs = [check_nrhs(r) for r in check_count(nrhs or [1] * n, n, "nrhs")]
        for o, p in zip(ops, pcs):
            if p is not None and p.op is not o:
                raise ValueError("a preconditioner was built for another operator")
        self._ops, self._pcs = list(ops), list(pcs)
        self.nrhs = list(nrhs)
        self.sizes = [o.n_active * r for o, r in zip(self._ops, self.nrhs)]
        oa = (C.c_void_p * n)(*[o._h.value for o in ops])
        pa = (C.c_void_p * n)(*[(p._h.value if p is not None else None) for p in pcs])
        ra = (C.c_int32 * n)(*nrhs)
        h_ = C.c_void_p()
        check(lib().cpm_batch_create(n, oa, pa, ra, C.byref(h_)))
        self._h = h_

    def solve(self, fs, us=None, opts: SolveOptions | None = None, stream=None, **kw):
        torch = _torch()
        opts = opts or SolveOptions(**kw)
        n = len(self._ops)
        fs = check_count(fs, n, "fs")
        us = [torch.zeros_like(f) for f in fs] if us is None else check_count(us, n, "us")
        for i, (f, u, m) in enumerate(zip(fs, us, self.sizes)):
            check_vec(f, m, f"fs[{i}]")
            check_vec(u, m, f"us[{i}]")
            check_disjoint(f, u, f"fs[{i}] and us[{i}]")
        fa = (C.c_void_p * n)(*[_dptr(f, m).value for f, m in zip(fs, self.sizes)])
        ua = (C.c_void_p * n)(*[_dptr(u, m).value for u, m in zip(us, self.sizes)])
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
        n = len(self._ops)
        xs = check_count(xs, n, "xs")
        ys = [torch.empty_like(x) for x in xs] if ys is None else check_count(ys, n, "ys")
        for i, (x, y, m) in enumerate(zip(xs, ys, self.sizes)):
            check_vec(x, m, f"xs[{i}]")
            check_vec(y, m, f"ys[{i}]")
            check_disjoint(x, y, f"xs[{i}] and ys[{i}]")
        xa = (C.c_void_p * n)(*[_dptr(x, m).value for x, m in zip(xs, self.sizes)])
        ya = (C.c_void_p * n)(*[_dptr(y, m).value for y, m in zip(ys, self.sizes)])
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
    a preconditioner built on A^T when one is given, and dL/dc comes from the
    library's fixed-order reduction (cpm_shift_gradient). Call as
    CPMSolve.apply(f, c, op, pc, pc_T, opts, adjoint_rtol) with c a 0-d tensor;
    adjoint_rtol (default opts.rtol) sets the A^T solve's tolerance, since the
    attainable residual of either solve is about eps |A| |u| / |f|.
    The operator's shift is set to c for each solve and restored afterwards;
    pc and pc_T keep the factors they were built with (built at another shift
    they are preconditioners of a nearby operator: the solution is unchanged,
    the iteration count may grow).
    """

    @staticmethod
    def forward(ctx, f, c, op, pc=None, pc_T=None, opts=None, adjoint_rtol=None):
        opts = opts or SolveOptions(rtol=1e-12)
        cval = float(c)
        with _shift(op, cval):
            u, st = solve(op, f.detach().contiguous(), pc=pc, opts=opts)
        if not st["converged"]:
            raise RuntimeError(f"forward solve did not converge: {st}")
        ctx.save_for_backward(u)
        ctx.op, ctx.pc_T, ctx.opts, ctx.c = op, pc_T, opts, cval
        ctx.adjoint_rtol = opts.rtol if adjoint_rtol is None else float(adjoint_rtol)
        ctx.c_meta = (c.device, c.dtype) if torch.is_tensor(c) else (u.device, u.dtype)
        return u

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        o = ctx.opts
        ot = SolveOptions(restart=o.restart, rtol=ctx.adjoint_rtol, atol=o.atol, max_it=o.max_it, mode="fp64",
                          transpose=True, stagnation_cycles=o.stagnation_cycles)
        with _shift(ctx.op, ctx.c):
            lam, st = solve(ctx.op, g.contiguous(), pc=ctx.pc_T, opts=ot)
        if not st["converged"]:
            raise RuntimeError(f"adjoint solve did not converge: {st}")
        gc = ctx.op.shift_gradient(lam, u)
        return lam, gc.reshape(()).to(device=ctx.c_meta[0], dtype=ctx.c_meta[1]), None, None, None, None, None


class _shift:
    """Sets an operator's shift for the duration of a block, then restores it."""

    def __init__(self, op: Operator, c: float):
        self.op, self.c = op, float(c)

    def __enter__(self):
        self.old = self.op.c
        if self.old != self.c:
            self.op.set_shift(self.c)
        return self.op

    def __exit__(self, *exc):
        if self.op.c != self.old:
            self.op.set_shift(self.old)
        return False


IMEX_SCHEME = {"euler": 0, "ark3": 1}
RD_KIND = {"gray_scott": 0, "heat": 1, "fitzhugh_nagumo": 2, "schnackenberg": 3}
# the paper's reaction parameters (Sec. 4.1.4: a, eps, beta; Sec. 4.1.6: d1, d2, lam)
RD_DEFAULTS = {"fitzhugh_nagumo": (0.1, 0.01, 0.5), "schnackenberg": (0.003, 0.7, 0.06)}


def imex_options(scheme="ark3", kind="gray_scott", dt=1.0, mu=(2e-5, 1e-5), F=0.04, k=0.06, tune=False, rd=None):
    o = _capi.ImexOpts()
    check(lib().cpm_imex_opts_default(C.byref(o)))
    o.scheme = IMEX_SCHEME[scheme]
    o.kind = RD_KIND[kind]
    o.nspecies = 1 if kind == "heat" else 2
    for q, val in enumerate(rd if rd is not None else RD_DEFAULTS.get(kind, (0.0, 0.0, 0.0))):
        o.rd[q] = float(val)
    o.dt = float(dt)
    for s, m in enumerate(tuple(mu)[:2]):
        o.mu[s] = float(m)
    o.F, o.k = float(F), float(k)
    o.tune = int(bool(tune))
    return o


def imex_shift(scheme="ark3", dt=1.0, mu=1.0) -> float:
    """The shift c = 1/(dt gamma mu) that a species' operator needs for the scheme's stage
    solves (gamma: the implicit tableau's diagonal), as the library defines it."""
    o = imex_options(scheme, "heat", dt, (mu, mu))
    c = float(lib().cpm_imex_shift(C.byref(o), 0))
    if not c > 0:
        raise ValueError("bad IMEX scheme, dt or mu")
    return c


class Imex:
    """Additive Runge-Kutta IMEX integrator of a surface reaction-diffusion system (ARK3(2)4L[2]SA
    or IMEX Euler), the stage solves batched over the species. ops: one operator per species at
    shift imex_shift(scheme, dt, mu_s); forcing (heat only): two device fields g1, g2 of the
    forcing cos(t) g1 + sin(t) g2."""

    def __init__(self, ops, pcs=None, scheme="ark3", kind="gray_scott", dt=1.0, mu=(2e-5, 1e-5), F=0.04, k=0.06,
                 forcing=None, tune=False, rd=None):
        self.opts = imex_options(scheme, kind, dt, mu, F, k, tune, rd)
        ns = self.opts.nspecies
        self._ops = check_count(ops, ns, "ops")
        self._pcs = check_count(pcs if pcs is not None else [None] * ns, ns, "pcs")
        self.n = self._ops[0].n_active
        for o, p in zip(self._ops, self._pcs):
            if o.n_active != self.n:
                raise ValueError("the species' operators must share one band")
            if p is not None and p.op is not o:
                raise ValueError("a preconditioner was built for another operator")
        oa = (C.c_void_p * ns)(*[o._h.value for o in self._ops])
        pa = (C.c_void_p * ns)(*[(p._h.value if p is not None else None) for p in self._pcs])
        fa = None
        if kind == "heat":
            forcing = check_count(forcing or [], 2, "forcing")
            fa = (C.c_void_p * 2)(*[_dptr(g, self.n, "forcing").value for g in forcing])
        h_ = C.c_void_p()
        check(lib().cpm_imex_create(oa, pa, C.byref(self.opts), fa, C.byref(h_)))
        self._h = h_

    def step(self, ws, t=0.0, nsteps=1, opts: SolveOptions | None = None, stream=None, **kw):
        """Advance the species' states ws (device vectors, in place) by nsteps steps from time t;
        returns one stats dict per species (summed over the stage solves)."""
        opts = opts or SolveOptions(**kw)
        ns = self.opts.nspecies
        ws = check_count(ws, ns, "ws")
        for i, w in enumerate(ws):
            check_vec(w, self.n, f"ws[{i}]")
        wa = (C.c_void_p * ns)(*[_dptr(w, self.n).value for w in ws])
        st = (_capi.SolveStats * ns)()
        co = opts.to_c()
        code = lib().cpm_imex_step(self._h, float(t), wa, int(nsteps), C.byref(co), st, _stream(stream))
        if code not in (_capi.CPM_OK, 6):
            check(code)
        return [_stats_dict(s) for s in st]

    def __del__(self):
        try:
            if getattr(self, "_h", None) is not None and self._h.value:
                lib().cpm_imex_destroy(self._h)
        except Exception:
            pass
