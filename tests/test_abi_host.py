"""Host-side tests of libctis: the shared library loads, exports every function
include/ctis.h declares, validates its inputs, and builds plan tables (box
grouping, support statistics, forward work list) that agree with brute force
and with the oracle's explicit H.  No GPU: plans are created host-only and no
compute call reaches a kernel."""
import ctypes
import os
import re
import zlib

import numpy as np
import pytest

from paper_2006_01573_amd import ctis, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctis.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ctis.LIB_PATH):
        from paper_2006_01573_amd import build
        build.build()
    return ctis.load_library()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctis_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_function(lib):
    names = header_functions()
    assert len(names) >= 12
    for nm in names:
        assert hasattr(lib, nm), f"libctis.so does not export {nm}"
    assert sorted(ctis.EXPORTED) == names


def test_status_strings_and_version(lib):
    for code in range(9):
        s = lib.ctis_status_str(code).decode()
        assert s and s != "unknown status"
    assert lib.ctis_status_str(99).decode() == "unknown status"
    assert re.fullmatch(r"\d+\.\d+\.\d+", lib.ctis_version().decode())


def host_plan(geo, ptr, idx, val, box=0, region=0):
    return ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val,
                     box=box, host_only=True, region=region)


def expect_status(code, fn, *a, **kw):
    with pytest.raises(ctis.CtisError) as ei:
        fn(*a, **kw)
    assert ei.value.status == code, str(ei.value)


def test_validation_errors(lib):
    geo = W.Geometry(3, 2, 2, 5, 4)
    ptr = np.array([0, 2, 3], np.int64)
    idx = np.array([0, 7, 19], np.int32)
    val = np.array([1.0, 0.5, 2.0], np.float32)
    host_plan(geo, ptr, idx, val)                                        # valid
    expect_status(1, ctis.Plan, 6, 2, 2, 5, 4, ptr, idx, val, host_only=True)   # a > gamma
    expect_status(1, ctis.Plan, 3, 5, 2, 5, 4, ptr, idx, val, host_only=True)   # alpha > xi
    expect_status(1, ctis.Plan, 3, 2, 2, 0, 4, ptr, idx, val, host_only=True)   # gamma = 0
    bad = idx.copy()
    bad[2] = 20
    expect_status(2, host_plan, geo, ptr, bad, val)                      # index == n
    bad[2] = -1
    expect_status(2, host_plan, geo, ptr, bad, val)
    badv = val.copy()
    badv[1] = np.inf
    expect_status(3, host_plan, geo, ptr, idx, badv)
    expect_status(1, host_plan, geo, np.array([0, 3, 2], np.int64), idx, val)   # decreasing
    expect_status(1, host_plan, geo, np.array([1, 2, 3], np.int64), idx, val)   # ptr[0] != 0
    expect_status(1, host_plan, geo, ptr, idx, val, box=9)
    expect_status(4, ctis.Plan, 1, 1, 1, 65536, 65536, np.array([0, 0], np.int64),
                  np.zeros(0, np.int32), np.zeros(0, np.float32), host_only=True)
    # unknown flag bits, through the raw ABI
    h = ctypes.c_void_p()
    st = lib.ctis_plan_create(ctypes.byref(h), 3, 2, 2, 5, 4, ctypes.c_void_p(ptr.ctypes.data),
                              ctypes.c_void_p(idx.ctypes.data), ctypes.c_void_p(val.ctypes.data), 0x10000)
    assert st == 1 and not h.value
    # region shape code 7 (CTIS_PLAN_REGION(7)) names no shape
    st = lib.ctis_plan_create(ctypes.byref(h), 3, 2, 2, 5, 4, ctypes.c_void_p(ptr.ctypes.data),
                              ctypes.c_void_p(idx.ctypes.data), ctypes.c_void_p(val.ctypes.data), 0x1 | (7 << 12))
    assert st == 1 and not h.value and "region shape" in lib.ctis_last_error().decode()
    assert lib.ctis_plan_create(None, 3, 2, 2, 5, 4, None, None, None, 1) == 1


def test_compute_on_host_only_plan_is_rejected(lib):
    geo = W.Geometry(3, 2, 1, 5, 4)
    p = host_plan(geo, np.array([0, 1], np.int64), np.array([3], np.int32), np.array([1.0], np.float32))
    dummy = ctypes.c_void_p(256)
    assert lib.ctis_forward(p._handle, dummy, ctypes.c_void_p(512), None) == 1
    assert lib.ctis_adjoint(p._handle, dummy, ctypes.c_void_p(512), None) == 1
    assert lib.ctis_em_iterate(p._handle, dummy, ctypes.c_void_p(512), 1, ctypes.c_void_p(1 << 20),
                               1 << 20, None) == 1
    assert "host-only" in lib.ctis_last_error().decode()
    assert lib.ctis_forward(None, dummy, dummy, None) == 1
    assert lib.ctis_em_iterate(p._handle, dummy, ctypes.c_void_p(512), -1, None, 0, None) == 1
    p.close()


def test_em_rejects_negative_plan_and_small_workspace(lib):
    geo = W.Geometry(3, 2, 1, 5, 4)
    p = host_plan(geo, np.array([0, 2], np.int64), np.array([3, 4], np.int32),
                  np.array([1.0, -0.5], np.float32))
    assert not p.info.nonnegative
    # negative check comes before the device check
    assert lib.ctis_em_iterate(p._handle, ctypes.c_void_p(256), ctypes.c_void_p(512), 1,
                               ctypes.c_void_p(1 << 20), 1 << 20, None) == 7
    q = host_plan(geo, np.array([0, 1], np.int64), np.array([3], np.int32), np.array([1.0], np.float32))
    assert lib.ctis_em_iterate(q._handle, ctypes.c_void_p(256), ctypes.c_void_p(512), 1,
                               ctypes.c_void_p(1 << 20), 4, None) == 8
    assert lib.ctis_em_iterate(q._handle, ctypes.c_void_p(256), ctypes.c_void_p(512), 1,
                               ctypes.c_void_p((1 << 20) + 4), 1 << 20, None) == 8


def reconstruct_calibration(plan, geo):
    """Dense c_s (float64) rebuilt from the plan's boxes."""
    lam, rc, vals = plan.boxes()
    B = plan.info.box
    c = np.zeros((geo.w, geo.n))
    for k in range(lam.size):
        for dc in range(B):
            for dr in range(B):
                v = vals[k, dc, dr]
                if v == 0.0:
                    continue
                r, cc = rc[k, 0] + dr, rc[k, 1] + dc
                assert 0 <= r < geo.gamma and 0 <= cc < geo.xi
                assert c[lam[k], r + geo.gamma * cc] == 0.0, "two boxes hold one position"
                c[lam[k], r + geo.gamma * cc] = v
    return c


CASES = [
    ("tiny-wrap", W.Geometry(3, 2, 3, 5, 4), 7, False),
    ("tiny-clustered", W.Geometry(4, 3, 2, 9, 7), 12, True),
    ("odd", W.Geometry(5, 7, 2, 13, 11), 9, True),
    ("a=gamma", W.Geometry(6, 2, 2, 6, 9), 5, False),
]


@pytest.mark.parametrize("name,geo,nnz,clustered", CASES)
@pytest.mark.parametrize("box", [0, 1, 2, 3, 5, 8])
def test_boxes_hold_exactly_the_merged_calibration(oracle_mod, lib, name, geo, nnz, clustered, box):
    rng = np.random.default_rng([zlib.crc32(name.encode()) % 1000, box])
    ptr, idx, val = W.random_kernels(geo, nnz, rng, clustered=clustered)
    idx[1] = idx[0]                       # a duplicate
    val[2] = 0.0                          # an explicit zero
    p = host_plan(geo, ptr, idx, val, box=box)
    if box:
        assert p.info.box == box
    c = reconstruct_calibration(p, geo)
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val, assemble=False)
    cp, ci, cv = o.calibration()
    ref = np.zeros((geo.w, geo.n))
    for s in range(geo.w):
        ref[s, ci[cp[s]:cp[s + 1]]] = cv[cp[s]:cp[s + 1]].astype(np.float32)
    np.testing.assert_array_equal(c, ref)
    assert p.info.nnz == int((ref != 0).sum())
    np.testing.assert_allclose(p.lambda_sums(), ref.sum(1), rtol=1e-6)


def brute_force_tiles(geo, B, rc, tile_fast, tile_slow):
    """FPA tiles met by one box's dilated image {(A + X + gamma*Y) mod n},
    X < a + B - 1, Y < alpha + B - 1 -- enumerated pixel by pixel."""
    ntr = -(-geo.gamma // tile_fast)
    A = int(rc[0]) + geo.gamma * int(rc[1])
    tiles = set()
    for Y in range(geo.alpha + B - 1):
        for X in range(geo.a + B - 1):
            i = (A + X + geo.gamma * Y) % geo.n
            r, c = i % geo.gamma, i // geo.gamma
            tiles.add(r // tile_fast + ntr * (c // tile_slow))
    return tiles


@pytest.mark.parametrize("name,geo,nnz,clustered", CASES + [
    ("wide", W.Geometry(40, 3, 2, 150, 40), 6, True),
    ("tall-wrap", W.Geometry(3, 20, 2, 70, 37), 6, False)])
def test_worklist_matches_brute_force(oracle_mod, lib, name, geo, nnz, clustered):
    rng = np.random.default_rng(zlib.crc32(name.encode()) % 10_000)
    ptr, idx, val = W.random_kernels(geo, nnz, rng, clustered=clustered)
    p = host_plan(geo, ptr, idx, val)
    inf = p.info
    lam, rc, _ = p.boxes()
    tp, ib = p.worklist()
    assert tp[0] == 0 and tp[-1] == inf.n_items and np.all(np.diff(tp) >= 0)
    got = {t: set(ib[tp[t]:tp[t + 1]].tolist()) for t in range(inf.n_tiles)}
    want = {t: set() for t in range(inf.n_tiles)}
    for k in range(inf.n_boxes):
        for t in brute_force_tiles(geo, inf.box, rc[k], inf.tile_fast, inf.tile_slow):
            want[t].add(k)
    assert got == want
    assert inf.n_active_tiles == sum(1 for t in want if want[t])
    # every pixel in a non-empty row of H sits in an active tile
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    _, rows, _ = o.csc()
    ntr = -(-geo.gamma // inf.tile_fast)
    for i in np.unique(rows):
        t = (i % geo.gamma) // inf.tile_fast + ntr * ((i // geo.gamma) // inf.tile_slow)
        assert got[t], f"support pixel {i} in an inactive tile"


@pytest.mark.parametrize("region", [0] + ctis.REGION_SHAPES[1:], ids=lambda r: f"{r[0]}x{r[1]}" if r else "default")
@pytest.mark.parametrize("name,geo,nnz,clustered", CASES + [
    ("margins", W.Geometry(23, 11, 3, 60, 44), 7, False),
    ("margins-clustered", W.Geometry(16, 12, 4, 64, 48), 9, True)])
def test_region_grid_matches_brute_force(oracle_mod, lib, name, geo, nnz, clustered, region):
    """The region path's grid (16 x 16 by default, every shape on request):
    the same cover rule as the tiles."""
    rng = np.random.default_rng(zlib.crc32(name.encode()) % 10_000 + 7)
    ptr, idx, val = W.random_kernels(geo, nnz, rng, clustered=clustered)
    p = host_plan(geo, ptr, idx, val, region=region)
    inf = p.info
    _, rc, _ = p.boxes()
    rp, ib = p.regions()
    assert (inf.region_fast, inf.region_slow) == (tuple(region) if region else (16, 16))
    assert rp[0] == 0 and rp[-1] == inf.n_region_items and np.all(np.diff(rp) >= 0)
    got = {t: set(ib[rp[t]:rp[t + 1]].tolist()) for t in range(inf.n_regions)}
    want = {t: set() for t in range(inf.n_regions)}
    for k in range(inf.n_boxes):
        for t in brute_force_tiles(geo, inf.box, rc[k], inf.region_fast, inf.region_slow):
            want[t].add(k)
    assert got == want
    assert inf.n_active_regions == sum(1 for t in want if want[t])
    # executed multiply-adds: B*B per box slot and output of every item
    BB = inf.box ** 2
    assert inf.region_forward_madds == inf.n_region_items * inf.region_fast * inf.region_slow * BB
    assert inf.tile_forward_madds == inf.n_items * inf.tile_fast * inf.tile_slow * BB
    assert inf.method_madds == geo.ell * inf.nnz


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_configurations_take_the_region_path(lib, cfg):
    """The configurations leave the margin the region path needs; there the
    region forward executes fewer multiply-adds than the tile forward."""
    case = W.make_case(cfg)
    p = ctis.Plan.from_case(case, host_only=True)
    inf = p.info
    assert inf.em_region_path
    ratio = inf.region_forward_madds / inf.method_madds
    assert ratio < inf.tile_forward_madds / inf.method_madds
    assert ratio <= {1: 4.5, 2: 1.9, 3: 1.4}[cfg]
    assert inf.adjoint_madds == inf.method_madds or cfg == 1   # the c1 field stop (16) is not a tile multiple


def test_region_path_needs_the_margin(lib):
    B = 3
    for gamma, xi, want in ((60 + 14 + B, 10 + 14 + B, True), (60 + 13 + B, 40, False), (90, 10 + 13 + B, False)):
        geo = W.Geometry(60, 10, 2, gamma, xi)
        ptr, idx, val = W.random_kernels(geo, 9, np.random.default_rng(5), clustered=True)
        p = host_plan(geo, ptr, idx, val, box=B)
        assert p.info.em_region_path == want, (gamma, xi)
    p = ctis.Plan(geo.a, geo.alpha, geo.w, 200, 200, ptr, idx, val, box=B, host_only=True, tile_path=True)
    assert not p.info.em_region_path


@pytest.mark.parametrize("name,geo,nnz,clustered", CASES)
def test_support_count_matches_explicit_H(oracle_mod, lib, name, geo, nnz, clustered):
    rng = np.random.default_rng(zlib.crc32(name.encode()) % 10_000 + 1)
    ptr, idx, val = W.random_kernels(geo, nnz, rng, clustered=clustered)
    p = host_plan(geo, ptr, idx, val)
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    _, rows, v = o.csc()
    assert p.info.n_support == np.unique(rows[v != 0]).size


def test_config_plans_c1_c2_c3(oracle_mod, lib):
    """The synthetic configurations group into exact blobs: 3x3 boxes (81 nnz
    per wavelength) for c1/c2, 5x5 boxes (625 per wavelength) for c3."""
    expect = {1: (3, 9, 5828), 2: (3, 9, 111744), 3: (5, 25, 730640)}
    for cfg, (B, per_lambda, n_supp) in expect.items():
        case = W.make_case(cfg)
        g = case.geometry
        p = host_plan(g, case.lambda_ptr, case.fpa_index, case.value)
        inf = p.info
        assert inf.box == B
        assert inf.n_boxes == per_lambda * g.w
        assert inf.nnz == case.value.size
        assert inf.n_support == n_supp
        assert inf.workspace_bytes >= 4 * g.n
        np.testing.assert_allclose(p.lambda_sums(),
                                   np.add.reduceat(case.value.astype(np.float64), case.lambda_ptr[:-1]),
                                   rtol=1e-6)


@pytest.mark.parametrize("box", [0, 1, 3, 5])
def test_keep_zeros_keeps_every_position_in_a_box(oracle_mod, lib, box):
    """With CTIS_PLAN_KEEP_ZEROS the structure is the set of given positions:
    an explicit zero and a duplicate pair that cancels stay inside boxes (as
    zero-valued slots); without it they are dropped and the plan says so."""
    geo = W.Geometry(9, 6, 3, 40, 30)
    rng = np.random.default_rng(box + 7)
    ptr, idx, val = W.random_kernels(geo, 14, rng, clustered=True)
    val[2] = 0.0
    idx[4] = idx[3]
    val[4] = -val[3]
    dropped = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val, box=box, host_only=True)
    kept = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val, box=box, host_only=True,
                     keep_zeros=True)
    assert dropped.info.dropped and not kept.info.dropped
    assert kept.info.n_entries == dropped.info.n_entries == int(ptr[-1])
    distinct = sum(np.unique(idx[ptr[s]:ptr[s + 1]]).size for s in range(geo.w))
    assert kept.info.nnz == distinct and dropped.info.nnz < distinct
    # the values are the merged calibration either way
    np.testing.assert_array_equal(reconstruct_calibration(kept, geo), reconstruct_calibration(dropped, geo))
    lam, rc, _ = kept.boxes()
    B = kept.info.box
    for s in range(geo.w):
        for i in idx[ptr[s]:ptr[s + 1]]:
            r, c = int(i) % geo.gamma, int(i) // geo.gamma
            inside = [(lam[k] == s and rc[k, 0] <= r < rc[k, 0] + B and rc[k, 1] <= c < rc[k, 1] + B)
                      for k in range(lam.size)]
            assert sum(inside) >= 1, (s, r, c)
    assert kept.info.vjp_workspace_bytes > kept.info.workspace_bytes > 0


def test_fourier_rejects_host_only_plans(lib):
    """The Fourier path needs a device plan: creating it from a host-only plan
    fails with CTIS_E_ARG before any device work."""
    import ctypes
    geo = W.Geometry(5, 4, 2, 16, 16)
    ptr, idx, val = W.random_kernels(geo, 5, np.random.default_rng(1))
    p = host_plan(geo, ptr, idx, val)
    h = ctypes.c_void_p()
    st = lib.ctis_fourier_create(ctypes.byref(h), p._handle)
    assert st == 1 and not h.value
    assert b"host-only" in lib.ctis_last_error()


def test_plan_refuses_an_unknown_region_shape(lib):
    geo = W.Geometry(3, 2, 2, 40, 40)
    ptr = np.array([0, 1, 2], np.int64)
    idx = np.array([0, 7], np.int32)
    val = np.array([1.0, 0.5], np.float32)
    for bad in [(12, 12), (16, 32), (4, 4)]:
        with pytest.raises(ValueError, match="region must be one of"):
            host_plan(geo, ptr, idx, val, region=bad)
    for good in ctis.REGION_SHAPES[1:]:
        assert (host_plan(geo, ptr, idx, val, region=good).info.region_fast,
                host_plan(geo, ptr, idx, val, region=good).info.region_slow) == good


def test_bench_refuses_more_than_one_gpu():
    """The measurement covers one GPU; asking for more exits with a message
    before anything touches a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("args,msg", [(["--region", "12x12"], "--region must be one of"),
                                      (["--region", "wide"], "--region must be one of"),
                                      (["--config", "4", "--c4-split", "5", "--c4-choice",
                                        "solo 32x8 W4 adjoint W1 Bauto"], "--c4-split takes"),
                                      (["--config", "4", "--c4-split", "2"], "--c4-split takes")])
def test_bench_refuses_bad_options_before_the_gpu(args, msg):
    """Malformed launch options exit with a message before anything touches a
    device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2, r.stderr
    assert msg in r.stderr
    assert r.stdout == ""


def test_tensor_arguments_are_checked_before_any_launch():
    """Every tensor the binding passes to the library by pointer goes through
    one validator (float32, contiguous, on the plan's device, exact element
    count), since the C side cannot check sizes."""
    torch = pytest.importorskip("torch")
    dev = torch.device("cpu")
    good = torch.zeros(12, dtype=torch.float32)
    assert ctis.need_tensor(good, 12, "f", dev) is good
    with pytest.raises(ValueError, match="12 elements"):
        ctis.need_tensor(torch.zeros(11), 12, "f", dev)
    with pytest.raises(ValueError, match="float32"):
        ctis.need_tensor(torch.zeros(12, dtype=torch.float64), 12, "f", dev)
    with pytest.raises(ValueError, match="contiguous"):
        ctis.need_tensor(torch.zeros(4, 6)[:, ::2], 12, "f", dev)
    with pytest.raises(ValueError, match="torch tensor"):
        ctis.need_tensor(np.zeros(12, np.float32), 12, "f", dev)
    with pytest.raises(ValueError, match="must be on"):
        ctis.need_tensor(good, 12, "f", torch.device("meta"))
    ws = torch.zeros(64)
    wp, wb = ctis.need_workspace(ws, 256, "workspace", dev)
    assert wb == 256 and wp.value == ws.data_ptr()
    with pytest.raises(ValueError, match="needs 260 bytes"):
        ctis.need_workspace(torch.zeros(64), 260, "workspace", dev)
    with pytest.raises(ValueError, match="contiguous"):
        ctis.need_workspace(torch.zeros(8, 16)[:, ::2], 16, "workspace", dev)
