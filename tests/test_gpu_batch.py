"""GPU parity of batches (many frames with their own plans in one launch per
kernel per EM iteration) against the FP64 oracle and against the
single-frame path."""
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


def test_uneven_batch_against_oracle(torch, ctis, oracle_mod):
    geos = [W.Geometry(5, 4, 3, 23, 17), W.Geometry(70, 6, 2, 90, 30), W.Geometry(3, 3, 4, 13, 11),
            W.Geometry(5, 4, 3, 23, 17)]
    rng = np.random.default_rng(77)
    kern = [W.random_kernels(g, 12, rng, clustered=True) for g in geos]
    kern[3] = kern[0]
    plans = [ctis.Plan(g.a, g.alpha, g.w, g.gamma, g.xi, *k, box=3) for g, k in zip(geos, kern)]
    plans[3] = plans[0]                        # a plan shared by two frames
    b = ctis.Batch(plans)
    orc = [oracle_mod.Oracle(g.a, g.alpha, g.w, g.gamma, g.xi, *k) for g, k in zip(geos, kern)]
    M, N = int(b.f_offsets[-1]), int(b.g_offsets[-1])
    f = rng.random(M).astype(np.float32)
    r = rng.random(N).astype(np.float32)
    g_all = b.forward(torch.from_numpy(f).cuda()).cpu().numpy()
    z_all = b.adjoint(torch.from_numpy(r).cuda()).cpu().numpy()
    fo, go = b.f_offsets, b.g_offsets
    for k in range(len(geos)):
        assert rel_l2(g_all[go[k]:go[k + 1]], orc[k].forward(f[fo[k]:fo[k + 1]])) <= PROJ_TOL
        assert rel_l2(z_all[fo[k]:fo[k + 1]], orc[k].adjoint(r[go[k]:go[k + 1]])) <= PROJ_TOL
    gim = np.concatenate([orc[k].forward(np.ones(g.m)) * rng.uniform(0.5, 1.5, g.n)
                          for k, g in enumerate(geos)]).astype(np.float32)
    fe = b.em(torch.from_numpy(gim).cuda(), 6).cpu().numpy()
    for k in range(len(geos)):
        assert rel_l2(fe[fo[k]:fo[k + 1]], orc[k].em(gim[go[k]:go[k + 1]], 6)) <= EM_TOL


@pytest.fixture(scope="module")
def c4(torch, ctis, oracle_mod):
    cfgs = W.batched_configs(64)
    cases = [W.make_case(4, frame=k, cfg=c) for k, c in enumerate(cfgs)]
    plans = [ctis.Plan.from_case(c) for c in cases]
    check = [0, 17, 63]
    orc = {k: oracle_mod.Oracle.from_case(cases[k]) for k in check}
    images = []
    for k, (c, p) in enumerate(zip(cases, plans)):
        if k in orc:
            clean = orc[k].forward(c.f_true.ravel())
        else:
            clean = p.forward(torch.from_numpy(c.f_true.astype(np.float32)).cuda()).double().cpu().numpy()
        images.append(c.noisy(clean))
    return cfgs, cases, plans, orc, images


def test_c4_batch_matches_single_frames_and_oracle(torch, ctis, c4):
    cfgs, cases, plans, orc, images = c4
    K = cfgs[0].iters
    log(f"c4: {len(plans)} frames, K={K}")
    b = ctis.Batch(plans)
    g_all = b.pack_g(images)
    f_all = b.em(g_all, K).cpu().numpy()
    worst = 0.0
    for k, p in enumerate(plans):
        single = p.em(torch.from_numpy(images[k]).cuda(), K).cpu().numpy().ravel()
        worst = max(worst, rel_l2(f_all[b.f_offsets[k]:b.f_offsets[k + 1]], single))
    log(f"c4 batch vs single-frame worst rel-L2 {worst:.2e}")
    assert worst <= 1e-5
    for k, o in orc.items():
        e = rel_l2(f_all[b.f_offsets[k]:b.f_offsets[k + 1]], o.em(images[k], K))
        log(f"c4 frame {k} vs oracle rel-L2 {e:.2e}")
        assert e <= EM_TOL
    assert np.all(f_all >= 0)


def test_batch_em_in_a_hip_graph(torch, ctis, c4):
    """The batched EM loop captured in a HIP graph and replayed several times,
    with eager work and synchronisations in between, reproduces the eager
    result every time."""
    cfgs, cases, plans, orc, images = c4
    b = ctis.Batch(plans[:16])
    g_all = b.pack_g(images[:16])
    ws = b.workspace()
    ref = b.em(g_all, 5, workspace=ws).clone()
    f_all = torch.ones_like(ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.em(g_all, 5, f_all=f_all, workspace=ws)          # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        f_all.fill_(1.0)
        b.em(g_all, 5, f_all=f_all, workspace=ws)
    for rep in range(3):
        junk = torch.rand(1 << 20, device="cuda").sum()     # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(f_all, ref), f"replay {rep} differs"
        del junk
