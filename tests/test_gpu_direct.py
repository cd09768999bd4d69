"""GPU parity of the direct window loads at their limits.

A forward window (64 + B - 1 by 16 + B - 1 positions of E f_s) is loaded as a
plain 2-D window over f_s bordered with zeros when the 1-D cyclic shift of
Sec. 3 cannot carry any position into the field stop: its origin lies
above a - gamma and alpha - xi and it ends inside the FPA.  A back-projection
window is loaded without wrapping when the box's image of the dilated field
stop stays inside the FPA and the last tile's window ends inside u.  The FPA
margins below sit one pixel under, at and one pixel over those limits, with
calibration nonzeros anywhere on the FPA (images that wrap round its end
included), for every box side; projections against the FP64 oracle at
relative L2 <= 1e-5, EM (tile path) at <= 1e-4.
"""
import sys

import numpy as np
import pytest

from paper_2006_01573_amd import workloads as W

pytestmark = pytest.mark.gpu

PROJ_TOL = 1e-5
EM_TOL = 1e-4


def rel_l2(x, ref):
    x = np.asarray(x, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    den = np.linalg.norm(ref)
    return np.linalg.norm(x - ref) / (den if den > 0 else 1.0)


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available(), "GPU tests need a visible MI355X"
    return _t


@pytest.fixture(scope="module")
def ctis(torch):
    from paper_2006_01573_amd import ctis as _c
    _c.load_library()
    return _c


CASES = [(box, d) for box in (1, 3, 5, 8) for d in (-1, 0, 1)]


@pytest.mark.parametrize("box,d", CASES, ids=[f"B{b}-margin{d:+d}" for b, d in CASES])
def test_direct_windows_at_their_limits(torch, ctis, oracle_mod, box, d):
    a, alpha, w = 20, 12, 3
    geo = W.Geometry(a, alpha, w, a + 64 + box - 1 + d, alpha + 16 + box - 1 + d)
    rng = np.random.default_rng(700 + 10 * box + d)
    kern = W.random_kernels(geo, 6 + box, rng, clustered=box % 2 == 1)
    print(f"direct limits B={box} margin {d:+d} geo={geo}", flush=True)
    sys.stdout.flush()
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern, box=box, tile_path=True)
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern)
    f = rng.uniform(0.2, 2.0, geo.m).astype(np.float32)
    r = rng.uniform(0.2, 2.0, geo.n).astype(np.float32)
    g = p.forward(torch.from_numpy(f).cuda()).cpu().numpy()
    z = p.adjoint(torch.from_numpy(r).cuda()).cpu().numpy()
    assert rel_l2(g, o.forward(f.astype(np.float64))) <= PROJ_TOL
    assert rel_l2(z, o.adjoint(r.astype(np.float64))) <= PROJ_TOL
    gim = (o.forward(np.ones(geo.m)) * rng.uniform(0.5, 1.5, geo.n)).astype(np.float32)
    fe = p.em(torch.from_numpy(gim).cuda(), 4).cpu().numpy()
    assert rel_l2(fe, o.em(gim, 4)) <= EM_TOL
