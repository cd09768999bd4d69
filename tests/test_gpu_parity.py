"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: relative L2 <= 1e-5 for one projection, <= 1e-4 after the full
iteration count of a configuration, float32 arithmetic on the GPU.  Inputs are
the same float32 values on both sides; the oracle promotes them to double.
"""
import ctypes
import sys
import zlib

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


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_plan(ctis, geo, ptr, idx, val, box=0):
    return ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val, box=box)


def oracle_for(oracle_mod, geo, ptr, idx, val, **kw):
    return oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val, **kw)


def check_projections(torch, ctis, oracle_mod, geo, ptr, idx, val, seed, box=0, signed=False):
    log(f"projections geo={geo} nnz={idx.size} box={box} seed={seed}")
    p = gpu_plan(ctis, geo, ptr, idx, val, box=box)
    o = oracle_for(oracle_mod, geo, ptr, idx, val)
    rng = np.random.default_rng(seed)
    f = rng.random(geo.m).astype(np.float32)
    r = rng.random(geo.n).astype(np.float32)
    if signed:
        f -= 0.5
        r -= 0.5
    g_gpu = p.forward(torch.from_numpy(f).cuda()).cpu().numpy()
    z_gpu = p.adjoint(torch.from_numpy(r).cuda()).cpu().numpy()
    g_ref = o.forward(f)
    z_ref = o.adjoint(r)
    eg, ez = rel_l2(g_gpu, g_ref), rel_l2(z_gpu, z_ref)
    # pixels no voxel projects to are exactly zero
    _, rows, _ = o.csc()
    off = np.ones(geo.n, bool)
    off[rows] = False
    assert np.all(g_gpu.ravel()[off] == 0.0)
    assert eg <= PROJ_TOL, f"forward rel-L2 {eg:.3e}"
    assert ez <= PROJ_TOL, f"adjoint rel-L2 {ez:.3e}"
    return p, o


EDGE = [
    ("c1-geometry-random", W.Geometry(16, 16, 8, 128, 128), 40, False),
    ("wrap-odd", W.Geometry(5, 7, 3, 13, 11), 9, False),
    ("tiny-fpa", W.Geometry(3, 2, 2, 5, 4), 6, False),            # FPA far smaller than a tile
    ("single-pixel", W.Geometry(1, 1, 4, 37, 29), 8, True),
    ("a=gamma", W.Geometry(70, 3, 2, 70, 41), 10, True),          # field stop fills FPA columns
    ("alpha=xi", W.Geometry(9, 33, 2, 67, 33), 10, True),
    ("ragged", W.Geometry(67, 19, 3, 203, 77), 25, True),         # several tiles + ragged tails
    ("wide", W.Geometry(130, 17, 2, 131, 64), 12, True),          # x tiles, gamma odd
]


@pytest.mark.parametrize("name,geo,nnz,clustered", EDGE, ids=[e[0] for e in EDGE])
def test_projection_parity_edge_cases(torch, ctis, oracle_mod, name, geo, nnz, clustered):
    rng = np.random.default_rng(zlib.crc32(name.encode()) % 99991)
    ptr, idx, val = W.random_kernels(geo, nnz, rng, clustered=clustered, nonneg=False)
    check_projections(torch, ctis, oracle_mod, geo, ptr, idx, val, seed=1, signed=True)


@pytest.mark.parametrize("box", [1, 2, 3, 4, 5, 6, 7, 8])
def test_projection_parity_every_box_size(torch, ctis, oracle_mod, box):
    geo = W.Geometry(21, 9, 3, 97, 61)
    rng = np.random.default_rng(100 + box)
    ptr, idx, val = W.random_kernels(geo, 30, rng, clustered=True)
    check_projections(torch, ctis, oracle_mod, geo, ptr, idx, val, seed=box, box=box)


# A window spans 16 + B - 1 FPA rows.  Where xi is at least that many rows
# the kernels take each row's offset by a wrap-once rule, below it row by
# row: xi one below, at and one above the window height, on FPAs narrower
# than a window (columns wrap onto the next row) and wider than one tile.
ROWS = [(box, dxi, cols) for box in range(1, 9) for dxi in (-1, 0, 1) for cols in ((11, 7), (70, 66))]


@pytest.mark.parametrize("box,dxi,cols", ROWS, ids=[f"B{b}-xi{15 + b + d}-g{c[0]}" for b, d, c in ROWS])
def test_window_rows_near_window_height(torch, ctis, oracle_mod, box, dxi, cols):
    gamma, a = cols
    xi = 15 + box + dxi
    geo = W.Geometry(a, min(xi, 5 + box), 2, gamma, xi)
    rng = np.random.default_rng(1000 * box + 10 * xi + gamma)
    ptr, idx, val = W.random_kernels(geo, 3 + box, rng, clustered=box % 2 == 0)
    p, o = check_projections(torch, ctis, oracle_mod, geo, ptr, idx, val, seed=box, box=box, signed=True)
    assert p.info.box == box
    g = (o.forward(rng.uniform(0.2, 2.0, geo.m)) * rng.uniform(0.7, 1.3, geo.n)).astype(np.float32)
    f = p.em(torch.from_numpy(g).cuda(), 2).cpu().numpy()
    assert rel_l2(f, o.em(g, 2)) <= EM_TOL


def test_empty_and_zero_wavelengths(torch, ctis, oracle_mod):
    geo = W.Geometry(8, 5, 3, 40, 30)
    # wavelength 1 has no entries, wavelength 2 only an explicit zero
    ptr = np.array([0, 3, 3, 4], np.int64)
    idx = np.array([5, 6, 200, 17], np.int32)
    val = np.array([1.0, 0.5, 0.25, 0.0], np.float32)
    p, o = check_projections(torch, ctis, oracle_mod, geo, ptr, idx, val, seed=7)
    g = torch.rand(geo.xi, geo.gamma, device="cuda")
    f = p.em(g, 3).cpu().numpy()
    ref = o.em(g.cpu().numpy(), 3)
    assert np.all(f[1] == 0) and np.all(f[2] == 0)
    assert rel_l2(f, ref) <= EM_TOL
    # no calibration entries at all
    p0 = gpu_plan(ctis, geo, np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    assert p0.info.n_active_tiles == 0
    assert torch.count_nonzero(p0.forward(torch.rand(p0.shape_f, device="cuda"))).item() == 0
    assert torch.count_nonzero(p0.adjoint(torch.rand(p0.shape_g, device="cuda"))).item() == 0
    assert torch.count_nonzero(p0.em(g, 2)).item() == 0


@pytest.fixture(scope="module")
def c1(torch, ctis, oracle_mod):
    case = W.make_case(1)
    o = oracle_mod.Oracle.from_case(case)
    g = case.noisy(o.forward(case.f_true.ravel()))
    p = ctis.Plan.from_case(case)
    return case, o, p, g


def test_c1_projections(torch, c1):
    case, o, p, _ = c1
    f = case.f_true.astype(np.float32)
    g_gpu = p.forward(torch.from_numpy(f).cuda()).cpu().numpy()
    assert rel_l2(g_gpu, o.forward(f)) <= PROJ_TOL
    r = np.random.default_rng(3).random(case.geometry.n).astype(np.float32)
    z_gpu = p.adjoint(torch.from_numpy(r).cuda()).cpu().numpy()
    assert rel_l2(z_gpu, o.adjoint(r)) <= PROJ_TOL


def test_c1_em_parity_and_invariants(torch, c1):
    case, o, p, g = c1
    K = case.cfg.iters
    log(f"c1 EM K={K}")
    f_gpu = p.em(torch.from_numpy(g).cuda(), K).cpu().numpy()
    f_ref = o.em(g, K)
    e = rel_l2(f_gpu, f_ref)
    log(f"c1 EM rel-L2 {e:.3e}")
    assert e <= EM_TOL
    assert np.all(f_gpu >= 0)
    h = np.repeat(p.lambda_sums().astype(np.float64), case.geometry.ell)
    flux = (h * f_gpu.ravel().astype(np.float64)).sum()
    np.testing.assert_allclose(flux, g.astype(np.float64).sum(), rtol=1e-5)


def test_em_from_the_adjoint_start(torch, ctis, c1):
    """The other start Sec. 2 names, f^(1) = H^T g: GPU EM from it against the
    oracle's EM from its own H^T g, for a plan and for a batch."""
    case, o, p, g = c1
    K = 10
    ref = o.em(g, K, f0=o.adjoint(g))
    gd = torch.from_numpy(g).cuda()
    e = rel_l2(p.em(gd, K, start="adjoint").cpu().numpy(), ref)
    log(f"c1 EM from H^T g: rel-L2 {e:.2e}")
    assert e <= EM_TOL
    b = ctis.Batch([p, p])
    fb = b.em(torch.cat([gd.reshape(-1), gd.reshape(-1)]), K, start="adjoint").cpu().numpy()
    assert rel_l2(fb[: case.geometry.m], ref) <= EM_TOL and rel_l2(fb[case.geometry.m:], ref) <= EM_TOL


def test_diagnostics_against_oracle(torch, ctis, oracle_mod, c1):
    """GPU diagnostics (flux, sum g, Poisson log-likelihood; double-precision
    reductions over the float projection) against the oracle's, at the start
    and after 5 EM iterations; a pixel with g > 0 that no voxel reaches makes
    the log-likelihood -inf."""
    case, o, p, g = c1
    gd = torch.from_numpy(g).cuda()
    for f in (np.ones(p.sizes.m, np.float32), p.em(gd, 5).cpu().numpy().ravel()):
        flux, sum_g, L, bad = p.diagnostics(gd, torch.from_numpy(f).cuda())
        fl_ref, L_ref = o.diagnostics(g, f)
        assert bad == 0
        assert abs(flux - fl_ref) <= 1e-6 * abs(fl_ref)
        assert abs(sum_g - float(np.sum(g, dtype=np.float64))) <= 1e-12 * sum_g
        assert abs(L - L_ref) <= 1e-6 * abs(L_ref)
    _, rows, _ = o.csc()
    off = np.setdiff1d(np.arange(p.sizes.n), rows)
    g2 = g.copy().ravel()
    g2[off[0]] = 1.0
    _, _, L, bad = p.diagnostics(torch.from_numpy(g2).cuda(), torch.ones(p.shape_f, device="cuda"))
    assert L == -np.inf and bad == 1


def test_adjoint_identity_gpu(torch, c1):
    case, o, p, _ = c1
    rng = np.random.default_rng(9)
    f = torch.from_numpy(rng.random(case.geometry.m).astype(np.float32) - 0.5).cuda()
    r = torch.from_numpy(rng.random(case.geometry.n).astype(np.float32) - 0.5).cuda()
    lhs = (p.forward(f).double() * r.view(p.shape_g).double()).sum().item()
    rhs = (f.view(p.shape_f).double() * p.adjoint(r).double()).sum().item()
    scale = (p.forward(f.abs()).double() * r.abs().view(p.shape_g).double()).sum().item()
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_fixed_point_noiseless_gpu(torch, c1, oracle_mod):
    case, o, p, _ = c1
    ft = (case.f_true + 1e-2).astype(np.float32)
    g = o.forward(ft).astype(np.float32)
    f = p.em(torch.from_numpy(g).cuda(), 20, f0=torch.from_numpy(ft).cuda()).cpu().numpy()
    assert rel_l2(f, ft) <= 1e-4


def test_determinism_and_resume(torch, c1):
    case, o, p, g = c1
    gd = torch.from_numpy(g).cuda()
    a = p.em(gd, 12)
    b = p.em(gd, 12)
    assert torch.equal(a, b)
    c = p.em(gd, 5)
    c = p.em(gd, 7, f=c)
    assert torch.equal(a, c)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d = p.em(gd, 12)
    s.synchronize()
    assert torch.equal(a, d)
    f = torch.rand(p.shape_f, device="cuda")
    assert torch.equal(p.forward(f), p.forward(f))


def test_gpu_error_paths(torch, ctis, c1):
    case, o, p, g = c1
    gd = torch.from_numpy(g).cuda()
    with pytest.raises(ValueError):
        p.forward(torch.zeros(5, device="cuda"))
    small = torch.empty(16, device="cuda")
    with pytest.raises(ValueError):                   # the binding checks sizes first
        p.em(gd, 1, workspace=small)
    # the library's own check of the workspace size
    f1 = torch.ones(p.shape_f, device="cuda")
    st = p._L.ctis_em_iterate(p._handle, ctypes.c_void_p(gd.data_ptr()), ctypes.c_void_p(f1.data_ptr()), 1,
                              ctypes.c_void_p(small.data_ptr()), ctypes.c_size_t(64),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 8
    neg = ctis.Plan(4, 4, 1, 16, 16, np.array([0, 2], np.int64), np.array([0, 3], np.int32),
                    np.array([1.0, -1.0], np.float32))
    with pytest.raises(ctis.CtisError) as ei:
        neg.em(torch.ones(16, 16, device="cuda"), 1)
    assert ei.value.status == 7
    # projections accept negative calibration values
    neg.forward(torch.ones(neg.shape_f, device="cuda"))
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def c2(torch, ctis, oracle_mod):
    case = W.make_case(2)
    o = oracle_mod.Oracle.from_case(case)
    g = case.noisy(o.forward(case.f_true.ravel()))
    p = ctis.Plan.from_case(case)
    return case, o, p, g


def test_c2_projections(torch, c2):
    case, o, p, _ = c2
    f = case.f_true.astype(np.float32)
    assert rel_l2(p.forward(torch.from_numpy(f).cuda()).cpu().numpy(), o.forward(f)) <= PROJ_TOL
    r = np.random.default_rng(4).random(case.geometry.n).astype(np.float32)
    assert rel_l2(p.adjoint(torch.from_numpy(r).cuda()).cpu().numpy(), o.adjoint(r)) <= PROJ_TOL


def test_c2_em_full_iterations(torch, c2):
    """The benchmark's workload and launch configuration: 100 iterations."""
    case, o, p, g = c2
    K = case.cfg.iters
    log(f"c2 EM K={K}")
    f_gpu = p.em(torch.from_numpy(g).cuda(), K).cpu().numpy()
    f_ref = o.em(g, K)
    e = rel_l2(f_gpu, f_ref)
    log(f"c2 EM rel-L2 {e:.3e}")
    assert e <= EM_TOL
    assert np.all(f_gpu >= 0)


@pytest.fixture(scope="module")
def largest_fpa(oracle_mod):
    """An FPA just below the 2^29-pixel limit (23170 x 23170), so byte
    offsets into g and u reach 2^31; a small datacube, spread-out nonzeros."""
    geo = W.Geometry(32, 32, 4, 23170, 23170)
    assert geo.n < 2 ** 29
    rng = np.random.default_rng(29)
    ptr, idx, val = W.random_kernels(geo, 6, rng)
    log(f"largest FPA: building the oracle for n = {geo.n}")
    o = oracle_for(oracle_mod, geo, ptr, idx, val)
    return geo, ptr, idx, val, o


@pytest.mark.parametrize("box", [0, 8])
def test_largest_fpa(torch, ctis, largest_fpa, box):
    geo, ptr, idx, val, o = largest_fpa
    rng = np.random.default_rng(30 + box)
    log(f"largest FPA box={box}: plan")
    p = gpu_plan(ctis, geo, ptr, idx, val, box=box)
    f = rng.random(geo.m).astype(np.float32)
    g = p.forward(torch.from_numpy(f).cuda()).cpu().numpy().ravel()
    g_ref = o.forward(f)
    nz = np.flatnonzero(g_ref)
    rows = np.concatenate([nz, rng.choice(geo.n, 4000, replace=False), np.arange(geo.n - geo.gamma, geo.n)])
    log(f"  forward: {nz.size} nonzero rows")
    assert rel_l2(g[rows], g_ref[rows]) <= PROJ_TOL
    assert not np.any(g[g_ref == 0])                   # pixels no voxel reaches stay 0
    del g
    r = rng.random(geo.n, dtype=np.float32)
    z = p.adjoint(torch.from_numpy(r).cuda()).cpu().numpy().ravel()
    assert rel_l2(z, o.adjoint(r)) <= PROJ_TOL
    del r
    gm = (g_ref * rng.uniform(0.7, 1.3, geo.n)).astype(np.float32)
    log("  EM, 2 iterations")
    fe = p.em(torch.from_numpy(gm).cuda(), 2).cpu().numpy()
    assert rel_l2(fe, o.em(gm, 2)) <= EM_TOL
    p.close()


def test_c3_sampled_projections(torch, ctis, oracle_mod):
    """Full-size c3 projections on the GPU, checked on sampled pixels and
    voxels that the oracle evaluates one by one from the definition."""
    case = W.make_case(3)
    geo = case.geometry
    log("c3 sampled projections")
    p = ctis.Plan.from_case(case)
    ok = oracle_mod.Oracle.from_case(case, assemble=False)
    rng = np.random.default_rng(33)
    f = case.f_true.astype(np.float32)
    g_gpu = p.forward(torch.from_numpy(f).cuda()).cpu().numpy().ravel()
    rows = rng.choice(geo.n, 3000, replace=False)
    rows = np.concatenate([rows, np.flatnonzero(g_gpu)[::997]])
    assert rel_l2(g_gpu[rows], ok.forward_rows(f, rows)) <= PROJ_TOL
    r = rng.random(geo.n).astype(np.float32)
    z_gpu = p.adjoint(torch.from_numpy(r).cuda()).cpu().numpy().ravel()
    cols = rng.choice(geo.m, 3000, replace=False)
    assert rel_l2(z_gpu[cols], ok.adjoint_cols(r, cols)) <= PROJ_TOL


def test_em_halves_compose_to_em_iterate(torch, c1):
    """ctis_em_forward_ratio + ctis_em_adjoint_update (out of place and in
    place) reproduce ctis_em_iterate bit for bit."""
    case, o, p, g = c1
    gd = torch.from_numpy(g).cuda()
    ref = p.em(gd, 3)
    f = torch.ones(p.shape_f, device="cuda")
    ws = p.workspace()
    tmp = torch.empty_like(f)
    for k in range(3):
        p.em_forward_ratio(f, gd, ws)
        if k % 2 == 0:
            p.em_adjoint_update(ws, f, tmp)
            f, tmp = tmp, f
        else:
            p.em_adjoint_update(ws, f, f)
    assert torch.equal(f, ref)


def test_c3_em_split_tiles_parity(torch, ctis, oracle_mod):
    """c3 geometry (FPA tiles with up to 273 boxes, back projection with 25
    boxes per wavelength): one EM iteration at full size against the
    oracle's single rows / columns (the ratio u is checked on sampled pixels,
    the update on sampled voxels)."""
    case = W.make_case(3)
    geo = case.geometry
    p = ctis.Plan.from_case(case)
    assert p.info.n_active_tiles < p._info().n_tiles
    log(f"c3 split: workspace {p.info.workspace_bytes} bytes")
    ok = oracle_mod.Oracle.from_case(case, assemble=False)
    rng = np.random.default_rng(5)
    f0 = (case.f_true + 0.05).astype(np.float32)
    g = (rng.random(geo.n) * 3).astype(np.float32)
    ws = p.workspace()
    fd = torch.from_numpy(f0).cuda()
    gd = torch.from_numpy(g).cuda()
    u = p.em_forward_ratio(fd, gd, ws).cpu().numpy().ravel()
    ghat = p.forward(fd).cpu().numpy().ravel()
    rows = np.flatnonzero(ghat > 0)[::61]
    gh_ref = ok.forward_rows(f0, rows)
    u_ref = g[rows].astype(np.float64) / gh_ref
    assert rel_l2(u[rows], u_ref) <= PROJ_TOL
    # a second pass on the same workspace
    u2 = p.em_forward_ratio(fd, gd, ws).cpu().numpy().ravel()
    assert np.array_equal(u, u2)
    f1 = p.em_adjoint_update(ws, fd, torch.empty_like(fd)).cpu().numpy().ravel()
    # the update needs u on the whole support: take it from the GPU's u only
    # through the oracle's own ratio on every support pixel
    cols = rng.choice(geo.m, 1500, replace=False)
    full_u = np.zeros(geo.n)
    sup = np.flatnonzero(ghat > 0)
    full_u[sup] = g[sup].astype(np.float64) / ok.forward_rows(f0, sup)
    zeta = ok.adjoint_cols(full_u, cols)
    h = np.repeat(p.lambda_sums().astype(np.float64), geo.ell)
    f1_ref = f0.ravel()[cols].astype(np.float64) * zeta / h[cols]
    assert rel_l2(f1[cols], f1_ref) <= PROJ_TOL


def test_split_tiles_em_parity(torch, ctis, oracle_mod):
    """70 wavelengths whose nonzeros all land near one spot: the FPA tiles
    there carry more boxes than one workgroup takes and are split; EM over
    several iterations (and repeated calls on one workspace) match the
    oracle."""
    geo = W.Geometry(8, 8, 70, 64, 40)
    rng = np.random.default_rng(11)
    ptr, idx, val = [0], [], []
    for s in range(geo.w):
        r, c = 20 + rng.integers(0, 4), 10 + rng.integers(0, 4)
        for dr in range(2):
            idx.append(r + dr + geo.gamma * c)
            val.append(rng.uniform(0.2, 1.0))
        ptr.append(len(idx))
    ptr, idx, val = np.array(ptr, np.int64), np.array(idx, np.int32), np.array(val, np.float32)
    p = gpu_plan(ctis, geo, ptr, idx, val)
    o = oracle_for(oracle_mod, geo, ptr, idx, val)
    assert p.info.workspace_bytes > 4 * geo.n + 256, "expected split tiles"
    g = (o.forward(np.ones(geo.m)) * rng.uniform(0.5, 1.5, geo.n)).astype(np.float32)
    gd = torch.from_numpy(g).cuda()
    ws = p.workspace()
    for k in (1, 4, 9):
        f = torch.ones(p.shape_f, device="cuda")
        p.em(gd, k, f=f, workspace=ws)
        assert rel_l2(f.cpu().numpy(), o.em(g, k)) <= EM_TOL
