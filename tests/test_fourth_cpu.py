"""Bands of reach 2 (the fourth-order stencil's ghost layer) through the C ABI on
the host: the library's Sigma_A, Sigma_G and closest points equal the oracle's
(sets keyed by grid index, closest points bit for bit), for cubic and quintic
interpolation, and the options are validated. No GPU call is made here."""
import numpy as np
import pytest

from oracle import fourth, surfaces
from paper_2110_06322_amd import _capi, cpm
from tests import gpu_cases as G


@pytest.mark.parametrize("kind,params,d,h,p", [("circle", (1.0,), 2, 0.05, 3), ("circle", (1.0,), 2, 0.05, 5),
                                               ("sphere", (1.0,), 3, 0.1, 3), ("sphere", (1.0,), 3, 0.1, 5),
                                               ("torus", (1.0, 0.4), 3, 0.05, 5)])
def test_reach2_band_matches_oracle(kind, params, d, h, p):
    G.ensure_built()
    lb = cpm.Band(kind, params, d, h, p, reach=2)
    ob = fourth.build_band_reach(surfaces.make_cp(kind, params), d, h, p, [-2.0] * d, [2.0] * d)
    assert lb.reach == 2
    assert lb.n_active == ob.n_active and lb.n_ghost == ob.n_ghost
    assert abs(lb.gamma - fourth.gamma_reach(d, p, h, 2)) <= 1e-15
    keys, pos = G.mapping(lb, ob)
    akeys, apos = G.all_mapping(lb, ob)
    _, cp, kd = lb.export()
    assert (kd[:lb.n_active] == 0).all() and (kd[lb.n_active:] == 1).all()
    assert np.array_equal(cp, ob.all_cp[apos])


def test_reach_and_degree_validation():
    G.ensure_built()
    with pytest.raises(_capi.CpmError):
        cpm.Band("sphere", (1.0,), 3, 0.1, 3, reach=3)
    with pytest.raises(_capi.CpmError):
        cpm.Band("sphere", (1.0,), 3, 0.1, 6)
    b1 = cpm.Band("sphere", (1.0,), 3, 0.1, 3)
    b2 = cpm.Band("sphere", (1.0,), 3, 0.1, 3, reach=2, gamma=b1.gamma)
    assert b1.reach == 1 and b2.reach == 2
    # same radius: the active set is the same or larger (closure over more ghosts), the ghosts grow
    assert b2.n_active >= b1.n_active and b2.n_ghost > b1.n_ghost
    assert set(b1.active_keys.tolist()) <= set(b2.active_keys.tolist())
