"""Open-surface bands built by the library on the host from a caller's closest point
callback (cpm_band_build_user) against the oracle's open band: equal active and
ghost sets, equal extension-row signs, interpolation points within a few ulp;
a failing callback is reported as CPM_ERR_ARG with the Python exception re-raised."""
import numpy as np
import pytest

from oracle import open_band as OB
from paper_2110_06322_amd import _capi, cpm, inputs, surfaces
from tests import gpu_cases as G

RIMS = {"neumann": None, "dirichlet": lambda phi: np.ones_like(phi, dtype=bool),
        "mixed": lambda phi: np.sin(3.0 * phi) < -0.5}


@pytest.mark.parametrize("rim", list(RIMS))
def test_callback_band_matches_oracle(rim):
    h = 0.1
    lb = cpm.Band.from_closest_point(surfaces.hemisphere(1.0, RIMS[rim]), 3, h, 3, [-1.6] * 3, [1.6] * 3)
    ob = OB.build_open_band(OB.hemisphere(RIMS[rim]), 3, h, 3, [-1.6] * 3, [1.6] * 3,
                            inputs.ruuth_merriman_gamma(3, 3, h))
    keys, pos = G.mapping(lb, ob)
    akeys, apos = G.all_mapping(lb, ob)
    assert lb.n_active == ob.n_active and lb.n_ghost == ob.ghost_keys.size and lb.n_band == ob.n_band
    ip, sg = lb.export_interp()
    assert np.array_equal(sg, ob.all_sign[apos])
    assert np.abs(ip - ob.all_ip[apos]).max() <= 8 * np.finfo(float).eps
    assert ((sg < 0).sum() > 0) == (rim != "neumann")


def test_closed_surface_interp_points_are_closest_points():
    b = cpm.Band("sphere", (1.0,), 3, 0.2, 3)
    _, cp, _ = b.export()
    ip, sg = b.export_interp()
    assert np.array_equal(ip, cp) and (sg == 1.0).all()


def test_failing_callback_raises():
    def bad(x):
        raise RuntimeError("surface unavailable")
    with pytest.raises(RuntimeError, match="surface unavailable"):
        cpm.Band.from_closest_point(bad, 3, 0.1, 3, [-1.6] * 3, [1.6] * 3)
