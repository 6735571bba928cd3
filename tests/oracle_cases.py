"""Cached oracle constructions shared by the tests (CPU, FP64)."""
from __future__ import annotations

import functools

import numpy as np

from oracle import band as B
from oracle import operator as O
from oracle import surfaces
from paper_2110_06322_amd import inputs

BOX2 = ([-2.0, -2.0], [2.0, 2.0])
BOX3 = ([-2.0, -2.0, -2.0], [2.0, 2.0, 2.0])


@functools.lru_cache(maxsize=None)
def band(kind: str, params: tuple, d: int, h: float, p: int, box=None):
    lo, hi = (BOX2 if d == 2 else BOX3) if box is None else box
    g = inputs.ruuth_merriman_gamma(d, p, h)
    pre = B.ellipsoid_prefilter(params, g) if kind == "ellipsoid" else None
    return B.build_band(surfaces.make_cp(kind, params), d, h, p, lo, hi, g, prefilter=pre)


@functools.lru_cache(maxsize=None)
def matrices(kind: str, params: tuple, d: int, h: float, p: int, c: float, box=None):
    bd = band(kind, params, d, h, p, box)
    E = O.assemble_E(bd)
    Om = O.assemble_O(bd)
    A = O.assemble_A(bd, c, E, Om)
    P = O.structural_pattern(bd, Om)
    return bd, E, Om, O.values_on_pattern(A, P), P


def circle_h005():
    """2-D unit circle, h = 0.05, p = 2, c = 1, f = (c+1) sin(theta(cp))."""
    return matrices("circle", (1.0,), 2, 0.05, 2, 1.0)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
