"""GPU parity of every region shape of the region forward (CTIS_PLAN_REGION
1..6: 8 x 32, 16 x 16, 32 x 8 with groups of 16 lanes, 16 x 8 and 8 x 16 with
groups of 8, 8 x 8 with groups of 4) against the FP64 oracle: the EM
forward half (u = g / H f) and EM iterations, on the cooperative kernel (the
groups of a wavefront share a region's boxes) and on the solo kernel (a
group per region), with random calibrations whose shifted images wrap round
the FPA (the 1-D cyclic shift of Sec. 3) in geometries that leave exactly
the margin each shape needs (and 5 pixels more), and with regions split
over several units (partial regions summed by a second kernel).
Tolerances: relative L2 <= 1e-5 for the forward half, <= 1e-4 after the
iterations.
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


SHAPES = [(8, 32), (16, 16), (32, 8), (16, 8), (8, 16), (8, 8)]
# (shape, B, extra margin): every shape at the smallest and largest box
# sides and one between, with the exact margin and a wider one
CASES = [(sh, box, extra) for sh in SHAPES for box, extra in ((1, 0), (3, 5), (5, 0), (8, 5))]


def ids(c):
    (rf, rs), box, extra = c
    return f"{rf}x{rs}-B{box}-m{extra}"


def geometry(shape, box, extra):
    rf, rs = shape
    a, alpha = 23, 11
    # the region path needs region + B - 2 pixels beside the field stop per axis
    return W.Geometry(a, alpha, 3, a + rf + box - 2 + extra, alpha + rs + box - 2 + 3 * extra)


def frame(oracle_mod, geo, kern, rng):
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern)
    g = (o.forward(rng.uniform(0.2, 2.0, geo.m)) * rng.uniform(0.7, 1.3, geo.n)).astype(np.float32)
    return o, g


@pytest.mark.parametrize("case", CASES, ids=[ids(c) for c in CASES])
def test_region_shape_em(torch, ctis, oracle_mod, case):
    shape, box, extra = case
    geo = geometry(shape, box, extra)
    rng = np.random.default_rng(1000 * box + 10 * shape[0] + shape[1] + extra)
    kern = W.random_kernels(geo, 4 + box, rng, clustered=(box + extra) % 2 == 1)
    log(f"region shape {shape} B={box} geo={geo}")
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern, box=box, region=shape)
    inf = p.info
    assert inf.box == box and inf.em_region_path and (inf.region_fast, inf.region_slow) == shape
    # one pixel less of margin on either axis: the tile path
    short = W.Geometry(geo.a, geo.alpha, geo.w, geo.gamma - extra - 1, geo.xi)
    ks = W.random_kernels(short, 4 + box, rng)
    assert not ctis.Plan(short.a, short.alpha, short.w, short.gamma, short.xi, *ks, box=box, region=shape,
                         host_only=True).info.em_region_path
    o, g = frame(oracle_mod, geo, kern, rng)
    gd = torch.from_numpy(g).cuda()
    f0 = rng.uniform(0.5, 1.5, geo.m).astype(np.float32)
    # forward half: u = g / (H f0) wherever some voxel projects
    u = p.em_forward_ratio(torch.from_numpy(f0).cuda(), gd, p.workspace()).cpu().numpy()
    gh = o.forward(f0.astype(np.float64))
    u_ref = np.where(gh > 0, g / np.where(gh > 0, gh, 1.0), 0.0)
    _, rows, _ = o.csc()
    sup = np.unique(rows)
    assert rel_l2(u.ravel()[sup], u_ref[sup]) <= PROJ_TOL
    ref = o.em(g, 3, f0=f0.astype(np.float64))
    f = p.em(gd, 3, f0=torch.from_numpy(f0).cuda()).cpu().numpy()
    assert rel_l2(f, ref) <= EM_TOL
    # the same frame twice with a lane group per region
    b = ctis.Batch([p, p], region_solo=True)
    assert b.info["em_region_path"] == 1
    fb = b.em(b.pack_g([g, g]), 3, f_all=torch.from_numpy(np.concatenate([f0, f0])).cuda()).cpu().numpy()
    fo = b.f_offsets
    assert rel_l2(fb[fo[0]:fo[1]], ref) <= EM_TOL
    assert rel_l2(fb[fo[1]:fo[2]], ref) <= EM_TOL


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{s[0]}x{s[1]}" for s in SHAPES])
def test_region_shape_split_regions(torch, ctis, oracle_mod, shape):
    """90 wavelengths whose nonzeros land near one spot: regions there carry
    more boxes than a unit takes and are split; the partial regions (of the
    shape's size, in slots of 256 floats) are summed by a second kernel.
    Both kernels against the oracle."""
    geo = W.Geometry(8, 8, 90, 64, 48)
    rng = np.random.default_rng(13 + shape[0] + 3 * shape[1])
    ptr, idx, val = [0], [], []
    for s in range(geo.w):
        r, c = 30 + rng.integers(0, 3), 20 + rng.integers(0, 3)
        for dr in range(2):
            idx.append(r + dr + geo.gamma * c)
            val.append(rng.uniform(0.2, 1.0))
        ptr.append(len(idx))
    kern = (np.array(ptr, np.int64), np.array(idx, np.int32), np.array(val, np.float32))
    log(f"split regions shape {shape}")
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern, region=shape)
    assert p.info.em_region_path and (p.info.region_fast, p.info.region_slow) == shape
    rp, _ = p.regions()
    assert np.diff(rp).max() > 64, "expected regions with more boxes than one unit takes"
    o, g = frame(oracle_mod, geo, kern, rng)
    gd = torch.from_numpy(g).cuda()
    ws = p.workspace()
    for k in (1, 4):
        f = torch.ones(p.shape_f, device="cuda")
        p.em(gd, k, f=f, workspace=ws)
        assert rel_l2(f.cpu().numpy(), o.em(g, k)) <= EM_TOL
    b = ctis.Batch([p], region_solo=True)
    f = b.em(gd, 4, workspace=b.workspace()).cpu().numpy()
    assert rel_l2(f, o.em(g, 4)) <= EM_TOL


@pytest.mark.parametrize("shape", [(16, 8), (8, 16), (8, 8)], ids=["16x8", "8x16", "8x8"])
def test_region_shape_c2_frame(torch, ctis, oracle_mod, shape):
    """The c2 frame (100 EM iterations) with the smaller regions, against
    the oracle, on both kernels (the solo one through a batch of the frame)."""
    case = W.make_case(2)
    o = oracle_mod.Oracle.from_case(case)
    g = case.noisy(o.forward(case.f_true.ravel()))
    gd = torch.from_numpy(g).cuda()
    log(f"c2 EM(100) shape {shape}")
    p = ctis.Plan.from_case(case, region=shape)
    assert p.info.em_region_path
    ref = o.em(g, 100)
    f = p.em(gd, 100).cpu().numpy()
    fs = ctis.Batch([p], region_solo=True).em(gd, 100).cpu().numpy()
    e, es = rel_l2(f, ref), rel_l2(fs, ref)
    log(f"  cooperative {e:.2e}, solo {es:.2e}")
    assert e <= EM_TOL and es <= EM_TOL


def test_batch_of_mixed_region_shapes_takes_the_tile_path(torch, ctis, oracle_mod):
    """Frames of one batch share the padded copy's border, so plans of
    different region shapes put the batch on the tile path; with one shape
    throughout it stays on the region path.  Both against the oracle."""
    geo = geometry((16, 16), 3, 5)
    rng = np.random.default_rng(77)
    kern = W.random_kernels(geo, 7, rng, clustered=True)
    o, g = frame(oracle_mod, geo, kern, rng)
    ref = o.em(g, 3)
    p16 = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern, box=3, region=(16, 16))
    p8 = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern, box=3, region=(8, 8))
    assert p16.info.em_region_path and p8.info.em_region_path
    for plans, region in (([p16, p8], 0), ([p8, p8], 1)):
        b = ctis.Batch(plans)
        assert b.info["em_region_path"] == region
        f = b.em(b.pack_g([g, g]), 3).cpu().numpy()
        fo = b.f_offsets
        for k in range(2):
            assert rel_l2(f[fo[k]:fo[k + 1]], ref) <= EM_TOL
