"""GPU parity of the other solvers on the same projections (simultaneous MART
and simultaneous nonnegative ART, ctis_solve_iterate) against the FP64
oracle's oracle_smart / oracle_sart, relative L2 <= 1e-4 after the iteration
count: on the region and the tile forward, with images that wrap round the
FPA, for uneven batches (cooperative and solo kernels), with SART's
relaxation below and above 1 and a calibration with negative values (SART
accepts any sign); and the error paths of the C ABI."""
import ctypes
import sys

import numpy as np
import pytest

from paper_2006_01573_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-4


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


def oracle_run(o, solver, g, iters, relax, f0=None):
    return o.smart(g, iters, f0=f0) if solver == "smart" else o.sart(g, iters, f0=f0, relax=relax)


@pytest.mark.parametrize("cfg,iters", [(1, 20), (2, 30)])
@pytest.mark.parametrize("solver,relax", [("smart", 1.0), ("sart", 1.0), ("sart", 0.6)])
@pytest.mark.parametrize("tile_path", [False, True], ids=["region", "tile"])
def test_solvers_match_oracle(torch, ctis, oracle_mod, cfg, iters, solver, relax, tile_path):
    case = W.make_case(cfg)
    o = oracle_mod.Oracle.from_case(case)
    g = case.noisy(o.forward(case.f_true.astype(np.float32).ravel()))
    p = ctis.Plan.from_case(case, tile_path=tile_path)
    assert bool(p.info.em_region_path) == (not tile_path)
    log(f"c{cfg} {solver} relax={relax} {'tile' if tile_path else 'region'} K={iters}")
    f = p.solve(torch.from_numpy(g).cuda(), iters, solver=solver, relax=relax).cpu().numpy()
    e = rel_l2(f, oracle_run(o, solver, g, iters, relax))
    log(f"  rel-L2 {e:.2e}")
    assert np.all(f >= 0)
    assert e <= TOL


WRAP = [(box, W.Geometry(11, 7, 3, 11 + 64 + box + 2, 7 + 16 + box + 3)) for box in (1, 3, 5, 8)]


@pytest.mark.parametrize("box,geo", WRAP, ids=[f"B{b}" for b, _ in WRAP])
def test_solvers_with_wrapping_images(torch, ctis, oracle_mod, box, geo):
    rng = np.random.default_rng(900 + box)
    kern = W.random_kernels(geo, 5 + box, rng, clustered=True)
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern)
    g = (o.forward(rng.uniform(0.2, 2.0, geo.m)) * rng.uniform(0.7, 1.3, geo.n)).astype(np.float32)
    gd = torch.from_numpy(g).cuda()
    for tile_path in (False, True):
        p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, *kern, box=box, tile_path=tile_path)
        for solver, relax in (("smart", 1.0), ("sart", 1.3)):
            f = p.solve(gd, 4, solver=solver, relax=relax).cpu().numpy()
            assert rel_l2(f, oracle_run(o, solver, g, 4, relax)) <= TOL, (tile_path, solver)


@pytest.mark.parametrize("kw", [{}, {"waves_adjoint": 1}, {"region_solo": True, "waves_adjoint": 1},
                                {"tile_path": True, "waves_forward": 1, "waves_adjoint": 1}],
                         ids=["cooperative", "solo-adjoint", "solo-region", "solo-tile"])
def test_batch_solvers_every_frame(torch, ctis, oracle_mod, kw):
    geos = [W.Geometry(16, 12, 4, 64, 48), W.Geometry(24, 20, 3, 80, 64), W.Geometry(16, 12, 4, 64, 48)]
    rng = np.random.default_rng(93)
    kern = [W.random_kernels(g, 9, rng, clustered=True) for g in geos]
    plans = [ctis.Plan(g.a, g.alpha, g.w, g.gamma, g.xi, *k, box=3) for g, k in zip(geos, kern)]
    b = ctis.Batch(plans, **kw)
    orc = [oracle_mod.Oracle(g.a, g.alpha, g.w, g.gamma, g.xi, *k) for g, k in zip(geos, kern)]
    gs = [(oc.forward(rng.uniform(0.2, 2.0, g.m)) * rng.uniform(0.7, 1.3, g.n)).astype(np.float32)
          for oc, g in zip(orc, geos)]
    g_all = b.pack_g(gs)
    ws = b.solve_workspace()
    fo = b.f_offsets
    for solver, relax in (("smart", 1.0), ("sart", 0.8)):
        f = b.solve(g_all, 6, solver=solver, relax=relax, workspace=ws).cpu().numpy()
        for k in range(len(geos)):
            assert rel_l2(f[fo[k]:fo[k + 1]], oracle_run(orc[k], solver, gs[k], 6, relax)) <= TOL, (solver, k)
    b.close()


def test_sart_with_negative_values(torch, ctis, oracle_mod):
    geo = W.Geometry(12, 9, 3, 50, 40)
    rng = np.random.default_rng(31)
    ptr, idx, val = W.random_kernels(geo, 8, rng)
    val = val.copy()
    val[::5] *= -0.3
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    g = (o.forward(rng.uniform(0.2, 2.0, geo.m)) + 0.5).astype(np.float32)
    f = p.solve(torch.from_numpy(g).cuda(), 5, solver="sart", relax=0.5).cpu().numpy()
    assert rel_l2(f, o.sart(g, 5, relax=0.5)) <= TOL
    with pytest.raises(ctis.CtisError):
        p.solve(torch.from_numpy(g).cuda(), 1, solver="smart")


def test_solver_error_paths(torch, ctis):
    case = W.make_case(1)
    p = ctis.Plan.from_case(case)
    L = p._L
    g = torch.ones(p.sizes.n, device="cuda")
    f = torch.ones(p.sizes.m, device="cuda")
    ws = p.solve_workspace()
    st = torch.cuda.current_stream().cuda_stream

    def call(solver, relax, nbytes, iters=1):
        return L.ctis_solve_iterate(p._handle, solver, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                    iters, ctypes.c_float(relax), ctypes.c_void_p(ws.data_ptr()), nbytes,
                                    ctypes.c_void_p(st))

    full = p.sizes.solve_workspace_bytes
    assert call(7, 1.0, full) == 1                                   # CTIS_E_ARG: unknown solver
    assert call(2, 2.5, full) == 1                                   # relax outside (0, 2)
    assert call(2, 0.0, full) == 1
    assert call(2, 1.0, full, iters=-1) == 1
    assert call(2, 1.0, p.sizes.workspace_bytes) == 8                # SART needs the larger workspace
    assert call(1, 1.0, p.sizes.workspace_bytes) == 0                # SMART fits in the EM workspace
    torch.cuda.synchronize()
    with pytest.raises(ValueError):
        p.solve(g, 1, solver="mart")


def test_solvers_degenerate_cases(torch, ctis, oracle_mod):
    """An empty wavelength (h = 0: its voxels go to 0), a single-pixel field
    stop, zero iterations (f untouched), and a frame of zeros (SMART keeps f,
    SART drives it to 0 within rounding)."""
    rng = np.random.default_rng(44)
    geo = W.Geometry(9, 7, 3, 40, 30)
    ptr, idx, val = W.random_kernels(geo, 6, rng)
    # drop wavelength 1's entries: it has no calibration (h = 0)
    ptr = ptr.copy()
    n1 = int(ptr[2] - ptr[1])
    keep = np.r_[np.arange(ptr[1]), np.arange(ptr[2], idx.size)]
    idx, val = idx[keep], val[keep]
    ptr[2:] -= n1
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    g = (o.forward(rng.uniform(0.2, 2.0, geo.m)) + 0.1).astype(np.float32)
    gd = torch.from_numpy(g).cuda()
    for solver in ("smart", "sart"):
        f = p.solve(gd, 3, solver=solver).cpu().numpy()
        assert np.all(f.reshape(geo.w, -1)[1] == 0.0)
        assert rel_l2(f, oracle_run(o, solver, g, 3, 1.0)) <= TOL
        f0 = torch.from_numpy(rng.uniform(0.5, 1.5, geo.m).astype(np.float32)).cuda()
        assert torch.equal(p.solve(gd, 0, solver=solver, f0=f0), f0)
    zeros = torch.zeros(geo.n, device="cuda")
    ones = p.solve(zeros, 2, solver="smart").cpu().numpy().reshape(geo.w, -1)
    assert np.all(ones[[0, 2]] == 1.0) and np.all(ones[1] == 0.0)
    # SART: r = -H f / R = -1 at f = 1, so one step reaches 0, up to FP32
    # rounding (H f and R = H 1 sum the same terms in different orders)
    assert np.abs(p.solve(zeros, 2, solver="sart").cpu().numpy()).max() <= 1e-6
    # a single-pixel field stop
    geo1 = W.Geometry(1, 1, 2, 13, 11)
    k1 = W.random_kernels(geo1, 5, rng)
    o1 = oracle_mod.Oracle(geo1.a, geo1.alpha, geo1.w, geo1.gamma, geo1.xi, *k1)
    p1 = ctis.Plan(geo1.a, geo1.alpha, geo1.w, geo1.gamma, geo1.xi, *k1)
    g1 = (o1.forward(np.array([0.7, 1.9])) * rng.uniform(0.8, 1.2, geo1.n)).astype(np.float32)
    for solver in ("smart", "sart"):
        f = p1.solve(torch.from_numpy(g1).cuda(), 5, solver=solver).cpu().numpy()
        assert rel_l2(f, oracle_run(o1, solver, g1, 5, 1.0)) <= TOL
