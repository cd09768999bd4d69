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
    """The 64 uneven frames of the batched workload, each with its frame made
    from the oracle's H f_true and its expected EM result from the oracle
    (one frame at a time, so that at most one explicit H is alive)."""
    cfgs = W.batched_configs(64)
    cases = [W.make_case(4, frame=k, cfg=c) for k, c in enumerate(cfgs)]
    plans = [ctis.Plan.from_case(c) for c in cases]
    K = cfgs[0].iters
    images, expected = [], []
    for k, c in enumerate(cases):
        o = oracle_mod.Oracle.from_case(c)
        images.append(c.noisy(o.forward(c.f_true.astype(np.float32).ravel())))
        expected.append(o.em(images[-1], K))
        o.close()
    log(f"c4: oracle results for {len(cases)} frames, K={K}")
    return cfgs, cases, plans, images, expected


def test_c4_batch_matches_oracle_every_frame(torch, ctis, c4):
    """All 64 frames of the batched solve (one launch per kernel per
    iteration, 50 iterations) against their own FP64 oracle solves, and
    against the single-frame path."""
    cfgs, cases, plans, images, expected = c4
    K = cfgs[0].iters
    b = ctis.Batch(plans)
    g_all = b.pack_g(images)
    f_all = b.em(g_all, K).cpu().numpy()
    assert np.all(f_all >= 0)
    errs = []
    for k in range(len(plans)):
        e = rel_l2(f_all[b.f_offsets[k]:b.f_offsets[k + 1]], expected[k])
        errs.append(e)
        assert e <= EM_TOL, f"frame {k} ({cfgs[k].name}) rel-L2 {e:.3e}"
    log(f"c4 vs oracle: worst rel-L2 {max(errs):.2e} (frame {int(np.argmax(errs))}), median {np.median(errs):.2e}")
    worst = 0.0
    for k, p in enumerate(plans):
        single = p.em(torch.from_numpy(images[k]).cuda(), K).cpu().numpy().ravel()
        worst = max(worst, rel_l2(f_all[b.f_offsets[k]:b.f_offsets[k + 1]], single))
    log(f"c4 batch vs single-frame worst rel-L2 {worst:.2e}")
    assert worst <= 1e-5


@pytest.mark.parametrize("path", ["tile", "region", "region_solo"])
def test_c4_solo_kernels_match_oracle_every_frame(torch, ctis, c4, path):
    """A wavefront per work unit (waves = 1: each wave walks all of its unit's
    boxes and writes its own micro-tiles) in the back projection, and in the
    forward projection on the tile path; on the region path with a lane group
    per region (four regions per wavefront); every frame against its oracle,
    also on a persistent grid."""
    cfgs, cases, plans, images, expected = c4
    K = cfgs[0].iters
    tile_path = path == "tile"
    for persistent in (False, True):
        kw = {"waves_forward": 1} if tile_path else {}
        b = ctis.Batch(plans, waves_adjoint=1, persistent=persistent, tile_path=tile_path,
                       region_solo=path == "region_solo", **kw)
        assert b.info["waves_adjoint"] == 1 and (not tile_path or b.info["waves_forward"] == 1)
        assert b.info["em_region_path"] == (0 if tile_path else 1)
        f_all = b.em(b.pack_g(images), K).cpu().numpy()
        worst = max(rel_l2(f_all[b.f_offsets[k]:b.f_offsets[k + 1]], expected[k]) for k in range(len(plans)))
        log(f"c4 solo {path} persistent={persistent}: worst rel-L2 {worst:.2e}")
        assert worst <= EM_TOL
        b.close()


def test_solo_projections_and_split_tiles(torch, ctis, oracle_mod):
    """Solo forward and back projections of uneven frames (one frame's FPA
    tiles carry more boxes than a unit takes, so they are split and summed by
    the second kernel) against the oracle, for every box side."""
    geo_hot = W.Geometry(8, 8, 90, 64, 48)
    rng = np.random.default_rng(21)
    ptr, idx, val = [0], [], []
    for s in range(geo_hot.w):
        r, c = 30 + rng.integers(0, 3), 20 + rng.integers(0, 3)
        for dr in range(2):
            idx.append(r + dr + geo_hot.gamma * c)
            val.append(rng.uniform(0.2, 1.0))
        ptr.append(len(idx))
    hot = (np.array(ptr, np.int64), np.array(idx, np.int32), np.array(val, np.float32))
    for box in (1, 3, 5, 8):
        geos = [W.Geometry(5, 4, 3, 23, 17), W.Geometry(70, 6, 2, 90, 30), geo_hot]
        kern = [W.random_kernels(g, 12, rng, clustered=True) for g in geos[:2]] + [hot]
        plans = [ctis.Plan(g.a, g.alpha, g.w, g.gamma, g.xi, *k, box=box) for g, k in zip(geos, kern)]
        b = ctis.Batch(plans, waves_forward=1, waves_adjoint=1, tile_path=True)
        orc = [oracle_mod.Oracle(g.a, g.alpha, g.w, g.gamma, g.xi, *k) for g, k in zip(geos, kern)]
        M, N = int(b.f_offsets[-1]), int(b.g_offsets[-1])
        f = rng.random(M).astype(np.float32)
        r = rng.random(N).astype(np.float32)
        log(f"solo projections B={box}")
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
        b.close()


@pytest.mark.parametrize("tile_path", [True, False], ids=["tile", "region"])
def test_batch_halves_compose_to_em_iterate(torch, ctis, c4, tile_path):
    """The two EM halves of a batch (forward + ratio, then back projection +
    update, which on the region path keeps the padded copy current) repeat
    ctis_batch_em_iterate bit for bit."""
    cfgs, cases, plans, images, _ = c4
    b = ctis.Batch(plans[:12], tile_path=tile_path)
    assert b.info["em_region_path"] == (0 if tile_path else 1)
    g_all = b.pack_g(images[:12])
    ref = b.em(g_all, 4)
    f = torch.ones(b.m_total, device="cuda")
    tmp = torch.empty_like(f)
    ws = b.workspace()
    for _ in range(4):
        b.em_forward_ratio(f, g_all, ws)
        b.em_adjoint_update(ws, f, tmp)
        f, tmp = tmp, f
    assert torch.equal(f, ref)


def test_tuned_batch_matches_oracle_every_frame(torch, ctis, c4):
    """The autotuned reconstruction (a configuration per frame shape: forward
    path, region shape, waves, persistent grid, box side; one batch per
    distinct choice) gives every one of the 64 frames its oracle result."""
    from paper_2006_01573_amd import tune
    cfgs, cases, plans, images, expected = c4
    K = cfgs[0].iters
    res = tune.autotune_frames(cases, images, iters=2, reps=1)
    log(f"c4 tuned: {res.classes}")
    assert sum(c["frames"] for c in res.classes) == len(cases)
    tb = res.batch
    f_all = tb.em(tb.pack_g(images), K)
    for k in range(len(cases)):
        e = rel_l2(tb.frame_f(f_all, k).cpu().numpy(), expected[k])
        assert e <= EM_TOL, f"frame {k} ({cfgs[k].name}, {res.classes}) rel-L2 {e:.3e}"
    tb.close()


def test_batch_em_in_a_hip_graph(torch, ctis, c4):
    """The batched EM loop captured in a HIP graph and replayed several times,
    with eager work and synchronisations in between, reproduces the eager
    result every time."""
    cfgs, cases, plans, images, _ = c4
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


@pytest.mark.parametrize("split", [2, 4])
def test_concurrent_batches_match_oracle_and_graph_replays(torch, ctis, c4, split):
    """The 64 frames as `split` batches of about equal work run side by side on
    streams of their own (one slice of the workspace each): every frame
    against its oracle, bit for bit the same batches run one after another,
    and the concurrent solve captured in a HIP graph reproduces the eager
    result on every replay (eager work and synchronisations in between)."""
    from paper_2006_01573_amd import tune
    cfgs, cases, plans, images, expected = c4
    K = cfgs[0].iters
    choice = tune.Choice.parse("solo 32x8 W4 adjoint W1 Bauto")
    tb = tune.fixed_frames(cases, choice, split=split)
    assert tb.concurrent and len(tb.groups) == split
    groups = [(ch, idx) for ch, idx, _, _, _, _ in tb.groups]
    seq = tune.TunedBatch(cases, groups, concurrent=False)
    assert seq.order == tb.order
    g_all = tb.pack_g(images)
    ws = tb.workspace()
    f_all = tb.em(g_all, K, workspace=ws)
    torch.cuda.synchronize()
    f_seq = seq.em(g_all, K)
    assert torch.equal(f_all, f_seq)
    worst = max(rel_l2(tb.frame_f(f_all, k).cpu().numpy(), expected[k]) for k in range(len(cases)))
    log(f"c4 {split} concurrent batches: worst rel-L2 {worst:.2e}")
    assert worst <= EM_TOL
    ref = f_all.clone()
    f_g = torch.ones_like(ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tb.em(g_all, 3, f_all=f_g, workspace=ws)           # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref3 = tb.em(g_all, 3, f_all=torch.ones_like(ref), workspace=ws).clone()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        f_g.fill_(1.0)
        tb.em(g_all, 3, f_all=f_g, workspace=ws)
    for rep in range(3):
        junk = torch.rand(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(f_g, ref3), f"replay {rep} differs"
        del junk
    with pytest.raises(ValueError):
        tb.em(g_all, 1, workspace=torch.empty(16, device="cuda"))
    tb.close()
    seq.close()


def test_concurrent_batches_of_different_launch_choices(torch, ctis, c4):
    """Per-shape groups with different kernels side by side (the 512^2 frames
    on the tile path, the 256^2 frames on the solo region path, a third group
    on the cooperative region path): every frame against its oracle and bit
    for bit the same groups run one after another."""
    from paper_2006_01573_amd import tune
    cfgs, cases, plans, images, expected = c4
    K = cfgs[0].iters
    small = [k for k, c in enumerate(cases) if c.geometry.gamma == 256]
    large = [k for k, c in enumerate(cases) if c.geometry.gamma != 256]
    groups = [(tune.Choice.parse("tile 64x16 W4 adjoint W1 Bauto"), large[::2]),
              (tune.Choice.parse("solo 32x8 W4 adjoint W1 Bauto"), small),
              (tune.Choice.parse("region 16x16 W3 adjoint Wauto Bauto"), large[1::2])]
    tb = tune.TunedBatch(cases, groups, concurrent=True)
    seq = tune.TunedBatch(cases, groups, concurrent=False)
    assert tb.concurrent and not seq.concurrent
    g_all = tb.pack_g(images)
    f_all = tb.em(g_all, K)
    f_seq = seq.em(g_all, K)
    torch.cuda.synchronize()
    assert torch.equal(f_all, f_seq)
    worst = max(rel_l2(tb.frame_f(f_all, k).cpu().numpy(), expected[k]) for k in range(len(cases)))
    log(f"c4 mixed concurrent groups: worst rel-L2 {worst:.2e}")
    assert worst <= EM_TOL
    tb.close()
    seq.close()
