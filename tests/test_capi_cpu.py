"""C-ABI library on the host: it loads, exports every symbol include/cpm.h
declares, and its band build matches the oracle's (sets keyed by grid index,
closest points bit for bit). No GPU call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2110_06322_amd import _capi, cpm, inputs
from tests import oracle_cases as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(_capi.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()


def header_functions():
    src = open(os.path.join(ROOT, "include", "cpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cpm_[A-Za-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 25
    L = ctypes.CDLL(_capi.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the binding declares exactly the header's functions
    assert sorted(n for n, _, _ in _capi.SIGNATURES) == names


def test_binding_structs_match_the_header_layout():
    L = _capi.lib()
    for i, st in enumerate(_capi.ABI_STRUCTS):
        assert L.cpm_abi_sizeof(i) == ctypes.sizeof(st), st.__name__
    assert L.cpm_abi_sizeof(len(_capi.ABI_STRUCTS)) == -1
    o = _capi.SolveOpts()
    assert L.cpm_solve_opts_default(ctypes.byref(o)) == 0
    assert o.poly_n == 0 and o.pc_power == 1 and o.restart == 30


def test_version_and_error_string():
    assert _capi.lib().cpm_version() == 1
    assert isinstance(_capi.lib().cpm_last_error(), bytes)


def _compare(kind, params, d, h, p):
    lib_band = cpm.Band(kind, params, d, h, p)
    ob = C.band(kind, params, d, h, p)
    g, cp, kd = lib_band.export()
    assert lib_band.n_active == ob.n_active and lib_band.n_ghost == ob.n_ghost
    assert lib_band.n_band == ob.n_band
    keys = np.zeros(g.shape[0], dtype=np.int64)
    for k in range(d):
        keys = keys * ob.shape[k] + g[:, k]
    ka, kg = keys[kd == 0], keys[kd == 1]
    assert (kd[:lib_band.n_active] == 0).all() and (kd[lib_band.n_active:] == 1).all()
    assert np.array_equal(np.sort(ka), ob.active_keys)
    assert np.array_equal(np.sort(kg), ob.ghost_keys)
    # closest points: identical IEEE operation order on both sides
    oa = np.searchsorted(ob.active_keys, ka)
    og = np.searchsorted(ob.ghost_keys, kg)
    ulp = np.spacing(np.maximum(np.abs(ob.cp_active[oa]), 1e-300))
    assert (np.abs(cp[kd == 0] - ob.cp_active[oa]) <= 4 * ulp).all()
    assert (np.abs(cp[kd == 1] - ob.cp_ghost[og]) <= 4 * np.spacing(np.maximum(np.abs(ob.cp_ghost[og]), 1e-300))).all()
    return lib_band, ob, cp[kd == 0], ob.cp_active[oa]


@pytest.mark.parametrize("kind,params,d,h,p", [
    ("circle", (1.0,), 2, 0.05, 2),
    ("circle", (1.0,), 2, 0.03, 3),
    ("sphere", (1.0,), 3, 0.1, 3),
    ("sphere", (1.0,), 3, 0.05, 2),
    ("torus", (1.0, 0.4), 3, 0.05, 3),
    ("ellipsoid", (1.3, 0.8, 0.65), 3, 0.05, 3),
])
def test_band_matches_oracle(kind, params, d, h, p):
    _, _, cl, co = _compare(kind, params, d, h, p)
    assert np.array_equal(cl, co) or kind == "ellipsoid"


def test_band_sphere_h002_sizes_and_bitwise_cp():
    lb, ob, cl, co = _compare("sphere", (1.0,), 3, 0.02, 3)
    assert (lb.n_band, lb.n_active, lb.n_ghost) == (260062, 187924, 52424)
    assert np.array_equal(cl, co)


def test_band_errors():
    with pytest.raises(_capi.CpmError) as e:
        cpm.Band("sphere", (1.0,), 3, 0.05, 3, lo=[-1.05] * 3, hi=[1.05] * 3)
    assert e.value.status == "CPM_ERR_BAND"
    for bad in [dict(kind="circle", params=(1.0,), d=3, h=0.1, p=3),
                dict(kind="sphere", params=(1.0,), d=3, h=-0.1, p=3),
                dict(kind="sphere", params=(1.0,), d=3, h=0.1, p=6),
                dict(kind="torus", params=(0.4, 1.0), d=3, h=0.1, p=3)]:
        with pytest.raises(_capi.CpmError) as e:
            cpm.Band(**bad)
        assert e.value.status == "CPM_ERR_ARG"


def test_band_reaching_the_medial_axis_is_rejected_by_both():
    """A coarse band around a flat ellipsoid covers its centre node, whose closest
    point is not unique: library and oracle both refuse to build it."""
    axes, box = (1.2410195721651176, 1.0657296288514941, 0.6753029137923193), ((-2.5,) * 3, (2.5,) * 3)
    with pytest.raises(_capi.CpmError) as e:
        cpm.Band("ellipsoid", axes, 3, 0.1, 3, lo=box[0], hi=box[1])
    assert e.value.status == "CPM_ERR_BAND" and "closest point" in str(e.value)
    with pytest.raises(ValueError):
        C.band("ellipsoid", axes, 3, 0.1, 3, box)


def test_gamma_default_matches_formula():
    b = cpm.Band("sphere", (1.0,), 3, 0.1, 3)
    assert abs(b.gamma - inputs.ruuth_merriman_gamma(3, 3, 0.1)) < 1e-15


def test_apply_work_plan_covers_every_tile_once(tmp_path):
    """The persistent apply's work plan (host code in the library): each work
    item goes to exactly one workgroup of its own XCD share, for cost-balanced
    and strided plans alike (a small C++ driver linked against the library)."""
    import shutil
    import subprocess
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    exe = str(tmp_path / "plan_pipe_check")
    src = os.path.join(ROOT, "tests", "cpp", "plan_pipe_check.cpp")
    lib_dir = os.path.dirname(_capi.LIB_PATH)
    subprocess.run(["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include", "-o", exe, src,
                    _capi.LIB_PATH, f"-Wl,-rpath,{lib_dir}"], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
