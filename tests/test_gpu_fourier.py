"""GPU parity of the Fourier (WBH) path -- projections and EM through
length-n FFTs -- against the FP64 oracle and against the gather path.

Tolerances: the FFT adds rounding of order log2(n) float ulps to each
projection (n <= 2^20: < 1e-6 relative), so the projection bound (1e-5) and
the EM bound after the configuration's iteration count (1e-4) are the same
as for the gather path.
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


EDGE = [
    ("tiny-odd-w", W.Geometry(5, 4, 3, 16, 16), 7, False, True),
    ("wrap", W.Geometry(9, 6, 4, 32, 64), 12, False, True),
    ("clustered", W.Geometry(16, 8, 2, 64, 32), 12, True, True),
    ("signed", W.Geometry(7, 5, 5, 32, 32), 9, False, False),
    ("a=gamma", W.Geometry(16, 3, 2, 16, 16), 5, False, True),
    # transform lengths 4, 8 and 512 x 256: the radix-4-only, single radix-8
    # and radix-4 + two radix-8 stage schedules
    ("n=16", W.Geometry(3, 2, 3, 4, 4), 5, False, True),
    ("n=64", W.Geometry(5, 7, 2, 8, 8), 5, False, True),
    ("n=2^17", W.Geometry(9, 6, 3, 512, 256), 5, True, True),
]


@pytest.mark.parametrize("name,geo,nnz,clustered,nonneg", EDGE, ids=[e[0] for e in EDGE])
def test_fourier_projections_edge_cases(torch, ctis, oracle_mod, name, geo, nnz, clustered, nonneg):
    rng = np.random.default_rng(zlib.crc32(name.encode()) % 1000)
    ptr, idx, val = W.random_kernels(geo, nnz, rng, clustered=clustered, nonneg=nonneg)
    log(f"fourier projections {name} geo={geo}")
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    F = ctis.Fourier(p)
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    f = rng.random(geo.m).astype(np.float32)
    r = rng.standard_normal(geo.n).astype(np.float32)
    ws = F.workspace()
    ws.fill_(float("nan"))
    g = F.forward(torch.from_numpy(f).cuda(), workspace=ws).cpu().numpy()
    z = F.adjoint(torch.from_numpy(r).cuda(), workspace=ws).cpu().numpy()
    assert rel_l2(g, o.forward(f)) <= PROJ_TOL
    assert rel_l2(z, o.adjoint(r)) <= PROJ_TOL


@pytest.mark.parametrize("cfg", [1, 2])
def test_fourier_em_against_oracle_and_gather(torch, ctis, oracle_mod, cfg):
    case = W.make_case(cfg)
    K = case.cfg.iters
    log(f"fourier EM c{cfg}, K={K}")
    o = oracle_mod.Oracle.from_case(case)
    g = case.noisy(o.forward(case.f_true.ravel()))
    p = ctis.Plan.from_case(case)
    F = ctis.Fourier(p)
    f = torch.from_numpy(case.f_true.astype(np.float32)).cuda()
    gf = F.forward(f).cpu().numpy()
    assert rel_l2(gf, o.forward(case.f_true.ravel())) <= PROJ_TOL
    assert rel_l2(gf, p.forward(f).cpu().numpy()) <= PROJ_TOL
    r = torch.from_numpy(g).cuda()
    assert rel_l2(F.adjoint(r).cpu().numpy(), o.adjoint(g)) <= PROJ_TOL
    fe = F.em(r, K).cpu().numpy()
    e = rel_l2(fe, o.em(g, K))
    log(f"  c{cfg} fourier EM vs oracle rel-L2 {e:.2e}")
    assert e <= EM_TOL
    assert np.all(fe >= 0) or np.abs(np.minimum(fe, 0)).max() <= 1e-6 * np.abs(fe).max()


def test_fourier_c3_sampled(torch, ctis, oracle_mod):
    """n = 2^20 (the four-step limit of 1024 x 1024): sampled rows and columns
    against the oracle's definition."""
    case = W.make_case(3)
    geo = case.geometry
    log("fourier c3 sampled projections")
    p = ctis.Plan.from_case(case)
    F = ctis.Fourier(p)
    assert F.info["n1"] == 1024 and F.info["n2"] == 1024
    ok = oracle_mod.Oracle.from_case(case, assemble=False)
    rng = np.random.default_rng(8)
    f = case.f_true.astype(np.float32)
    g = F.forward(torch.from_numpy(f).cuda()).cpu().numpy().ravel()
    rows = np.concatenate([rng.choice(geo.n, 2000, replace=False), np.flatnonzero(g > 1e-3 * g.max())[::401]])
    assert rel_l2(g[rows], ok.forward_rows(f, rows)) <= PROJ_TOL
    r = rng.random(geo.n).astype(np.float32)
    z = F.adjoint(torch.from_numpy(r).cuda()).cpu().numpy().ravel()
    cols = rng.choice(geo.m, 2000, replace=False)
    assert rel_l2(z[cols], ok.adjoint_cols(r, cols)) <= PROJ_TOL


def test_fourier_error_paths(torch, ctis):
    geo = W.Geometry(5, 4, 2, 24, 16)                 # n = 384: not a power of two
    ptr, idx, val = W.random_kernels(geo, 5, np.random.default_rng(1))
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    with pytest.raises(ctis.CtisError) as ei:
        ctis.Fourier(p)
    assert ei.value.name == "CTIS_E_ARG"
    geo = W.Geometry(5, 4, 2, 16, 16)
    ptr, idx, val = W.random_kernels(geo, 5, np.random.default_rng(1))
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    F = ctis.Fourier(p)
    small = torch.empty(16, device="cuda")
    f1 = torch.ones(p.shape_f, device="cuda")
    out = torch.empty(p.shape_g, device="cuda")
    with pytest.raises(ValueError):                   # the binding checks sizes first
        F.forward(f1, workspace=small)
    # the library's own check of the workspace size
    st = F._L.ctis_fourier_forward(F._handle, ctypes.c_void_p(f1.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(small.data_ptr()), ctypes.c_size_t(64),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert ctis.STATUS_NAMES[st] == "CTIS_E_WORKSPACE"
    val2 = val.copy()
    val2[0] = -1.0
    F2 = ctis.Fourier(ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val2))
    with pytest.raises(ctis.CtisError) as ei:
        F2.em(torch.ones(p.shape_g, device="cuda"), 1)
    assert ei.value.name == "CTIS_E_NEGATIVE"
