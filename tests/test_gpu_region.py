"""GPU parity of the region path of the EM iteration (16 x 16 FPA regions,
four boxes per wavefront, windows read from a zero-bordered copy of f)
against the FP64 oracle and against the tile path.

The region path applies where the FPA leaves 14 + B pixels beside the field
stop on both axes; there the host writes every window origin inside the
padded block, also for shifted images that run past an FPA edge (the 1-D
cyclic shift of Sec. 3), which the random calibrations below produce.
Tolerances as for the other EM tests: relative L2 <= 1e-5 for one forward
half (the ratio u), <= 1e-4 after the iteration count.
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


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


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


def frame(oracle_mod, geo, kern, rng):
    """Oracle and a frame g = H f_true modulated by noise-like factors."""
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern)
    g = (o.forward(rng.uniform(0.2, 2.0, geo.m)) * rng.uniform(0.7, 1.3, geo.n)).astype(np.float32)
    return o, g


def ratio_ref(o, g, f):
    """u = g / (H f), 0 where H f <= 0 (Sec. 3 algorithm, ratio step)."""
    gh = o.forward(f)
    return np.where(gh > 0, g / np.where(gh > 0, gh, 1.0), 0.0)


# geometries with the margins, random calibrations anywhere on the FPA (their
# shifted images cross the FPA's last row and its end), every box side
WRAP = [(box, W.Geometry(23, 11, 3, 23 + 14 + box + extra, 11 + 14 + box + 3 * extra))
        for box in range(1, 9) for extra in (0, 5)]


@pytest.mark.parametrize("box,geo", WRAP, ids=[f"B{b}-g{g.gamma}-xi{g.xi}" for b, g in WRAP])
def test_region_em_with_wrapping_images(torch, ctis, oracle_mod, box, geo):
    rng = np.random.default_rng(50 * box + geo.gamma)
    kern = W.random_kernels(geo, 4 + box, rng, clustered=box % 2 == 1)
    log(f"region wrap B={box} geo={geo}")
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern, box=box)
    assert p.info.box == box and p.info.em_region_path
    o, g = frame(oracle_mod, geo, kern, rng)
    gd = torch.from_numpy(g).cuda()
    f0 = rng.uniform(0.5, 1.5, geo.m).astype(np.float32)
    ws = p.workspace()
    u = p.em_forward_ratio(torch.from_numpy(f0).cuda(), gd, ws).cpu().numpy()
    u_ref = ratio_ref(o, g, f0.astype(np.float64))
    # the back projection reads u only where some voxel projects
    _, rows, _ = o.csc()
    sup = np.unique(rows)
    assert rel_l2(u.ravel()[sup], u_ref[sup]) <= PROJ_TOL
    f = p.em(gd, 3, f0=torch.from_numpy(f0).cuda()).cpu().numpy()
    assert rel_l2(f, o.em(g, 3, f0=f0.astype(np.float64))) <= EM_TOL


@pytest.mark.parametrize("box,geo", WRAP[::3], ids=[f"B{b}-g{g.gamma}-xi{g.xi}" for b, g in WRAP[::3]])
def test_solo_regions_with_wrapping_images(torch, ctis, oracle_mod, box, geo):
    """A lane group per region (a batch of the frame and a second frame,
    region_solo), with images that wrap round the FPA: EM against the
    oracle."""
    rng = np.random.default_rng(60 * box + geo.xi)
    kern = W.random_kernels(geo, 4 + box, rng, clustered=box % 2 == 0)
    log(f"solo regions wrap B={box} geo={geo}")
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern, box=box)
    b = ctis.Batch([p, p], region_solo=True)
    assert b.info["em_region_path"] == 1
    o, g1 = frame(oracle_mod, geo, kern, rng)
    _, g2 = frame(oracle_mod, geo, kern, rng)
    f = b.em(b.pack_g([g1, g2]), 3).cpu().numpy()
    fo = b.f_offsets
    assert rel_l2(f[fo[0]:fo[1]], o.em(g1, 3)) <= EM_TOL
    assert rel_l2(f[fo[1]:fo[2]], o.em(g2, 3)) <= EM_TOL


def test_region_and_tile_paths_agree_c2(torch, ctis, oracle_mod):
    """The c2 frame (100 EM iterations) on both paths, each against the oracle."""
    case = W.make_case(2)
    o = oracle_mod.Oracle.from_case(case)
    g = case.noisy(o.forward(case.f_true.ravel()))
    gd = torch.from_numpy(g).cuda()
    pr = ctis.Plan.from_case(case)
    pt = ctis.Plan.from_case(case, tile_path=True)
    assert pr.info.em_region_path and not pt.info.em_region_path
    fr = pr.em(gd, 100).cpu().numpy()
    ft = pt.em(gd, 100).cpu().numpy()
    ref = o.em(g, 100)
    er, et = rel_l2(fr, ref), rel_l2(ft, ref)
    log(f"c2 EM(100): region {er:.2e}, tile {et:.2e}, region vs tile {rel_l2(fr, ft):.2e}")
    assert er <= EM_TOL and et <= EM_TOL


def test_split_regions(torch, ctis, oracle_mod):
    """90 wavelengths whose nonzeros land near one spot: the regions there
    carry more boxes than a unit takes and are split (partial regions summed
    by a second kernel); EM matches the oracle, repeatedly on one workspace."""
    geo = W.Geometry(8, 8, 90, 64, 48)
    rng = np.random.default_rng(12)
    ptr, idx, val = [0], [], []
    for s in range(geo.w):
        r, c = 30 + rng.integers(0, 3), 20 + rng.integers(0, 3)
        for dr in range(2):
            idx.append(r + dr + geo.gamma * c)
            val.append(rng.uniform(0.2, 1.0))
        ptr.append(len(idx))
    kern = (np.array(ptr, np.int64), np.array(idx, np.int32), np.array(val, np.float32))
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern)
    assert p.info.em_region_path
    rp, _ = p.regions()
    assert np.diff(rp).max() > 64, "expected regions with more boxes than one unit takes"
    o, g = frame(oracle_mod, geo, kern, rng)
    gd = torch.from_numpy(g).cuda()
    ws = p.workspace()
    for k in (1, 4, 7):
        f = torch.ones(p.shape_f, device="cuda")
        p.em(gd, k, f=f, workspace=ws)
        assert rel_l2(f.cpu().numpy(), o.em(g, k)) <= EM_TOL
    # the same with a lane group per region (split chunks write partial regions)
    b = ctis.Batch([p], region_solo=True)
    wsb = b.workspace()
    for k in (1, 4):
        f = b.em(gd, k, workspace=wsb).cpu().numpy()
        assert rel_l2(f, o.em(g, k)) <= EM_TOL


def test_region_halves_compose_to_em_iterate(torch, ctis):
    """Forward half (padded copy + projection) and update half (which keeps the
    padded copy current) reproduce ctis_em_iterate bit for bit."""
    case = W.make_case(1)
    p = ctis.Plan.from_case(case)
    assert p.info.em_region_path
    g = torch.from_numpy(case.noisy(np.ones(p.sizes.n))).cuda()
    ref = p.em(g, 4)
    f = torch.ones(p.shape_f, device="cuda")
    tmp = torch.empty_like(f)
    ws = p.workspace()
    for k in range(4):
        p.em_forward_ratio(f, g, ws)
        p.em_adjoint_update(ws, f, tmp)
        f, tmp = tmp, f
    assert torch.equal(f, ref)


def test_region_batch_matches_frames(torch, ctis, oracle_mod):
    """Uneven frames (with margins) in one batch on the region path: every
    frame against its oracle, and the batch against the tile-path batch."""
    geos = [W.Geometry(16, 12, 4, 64, 48), W.Geometry(24, 20, 3, 80, 64), W.Geometry(16, 12, 4, 64, 48)]
    rng = np.random.default_rng(91)
    kern = [W.random_kernels(g, 9, rng, clustered=True) for g in geos]
    plans = [ctis.Plan(g.a, g.alpha, g.w, g.gamma, g.xi, *k, box=3) for g, k in zip(geos, kern)]
    b = ctis.Batch(plans)
    bt = ctis.Batch(plans, tile_path=True)
    assert b.info["em_region_path"] == 1 and bt.info["em_region_path"] == 0
    orc, gs = zip(*[frame(oracle_mod, g, k, rng) for g, k in zip(geos, kern)])
    g_all = b.pack_g(gs)
    f = b.em(g_all, 5).cpu().numpy()
    ft = bt.em(g_all, 5).cpu().numpy()
    fo = b.f_offsets
    for k in range(len(geos)):
        assert rel_l2(f[fo[k]:fo[k + 1]], orc[k].em(gs[k], 5)) <= EM_TOL
    assert rel_l2(f, ft) <= 1e-5
