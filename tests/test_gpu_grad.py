"""GPU parity of the EM derivatives (ctis_em_vjp, ctis_batch_em_vjp, the value
updates and the unrolled autograd Function) against the FP64 oracle.

Tolerances (relative L2 over the compared vector):
  * one step, dL/df: four FP32 projections with FP32 accumulation, like the
    plain projections -> 1e-5;
  * one step, dL/dv: each value derivative sums u b + e f over all voxels of
    a wavelength (thousands of terms of both signs) -> 1e-4;
  * K unrolled steps (gradients of f0 and of the values): the stated bound for
    results after the iteration count -> 1e-4.
"""
import sys

import numpy as np
import pytest

from paper_2006_01573_amd import workloads as W

pytestmark = pytest.mark.gpu

DF_TOL = 1e-5
DV_TOL = 1e-4
GRAD_TOL = 1e-4


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


def split_case():
    # 70 wavelengths whose nonzeros sit near one spot: FPA tiles with more
    # than 64 boxes, split over several workgroups
    geo = W.Geometry(8, 8, 70, 64, 40)
    rng = np.random.default_rng(11)
    ptr, idx, val = [0], [], []
    for _ in range(geo.w):
        r, c = 20 + rng.integers(0, 4), 10 + rng.integers(0, 4)
        for dr in range(2):
            idx.append(r + dr + geo.gamma * c)
            val.append(rng.uniform(0.2, 1.0))
        ptr.append(len(idx))
    return geo, np.array(ptr, np.int64), np.array(idx, np.int32), np.array(val, np.float32)


def edge_cases():
    out = []
    geo = W.Geometry(5, 7, 3, 13, 11)
    ptr, idx, val = W.random_kernels(geo, 9, np.random.default_rng(3))
    first = slice(ptr[0], ptr[1])
    val[first][idx[first] == idx[4]] = 0.0          # a position whose value is 0, kept as structure
    out.append(("wrap-odd-zero", geo, ptr, idx, val, 0))
    for B in range(1, 9):
        geo = W.Geometry(9, 6, 2, 40, 30)
        ptr, idx, val = W.random_kernels(geo, 14, np.random.default_rng(B), clustered=True)
        out.append((f"box{B}", geo, ptr, idx, val, B))
    geo = W.Geometry(70, 20, 3, 90, 64)           # two field-stop tiles, a ragged tail
    ptr, idx, val = W.random_kernels(geo, 12, np.random.default_rng(21), clustered=True)
    out.append(("ragged", geo, ptr, idx, val, 0))
    out.append(("split",) + split_case() + (0,))
    for B in range(1, 9):                          # xi equal to the window height 16 + B - 1
        geo = W.Geometry(7, 5 + B, 2, 11, 15 + B)
        ptr, idx, val = W.random_kernels(geo, 3 + B, np.random.default_rng(40 + B), clustered=True)
        out.append((f"rows-box{B}", geo, ptr, idx, val, B))
    return out


def problem(oracle_mod, geo, ptr, idx, val, seed):
    rng = np.random.default_rng(seed)
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val.astype(np.float64))
    f = rng.uniform(0.5, 1.5, geo.m).astype(np.float32)
    g = (o.forward(rng.uniform(0.2, 2.0, geo.m)) * rng.uniform(0.7, 1.3, geo.n)).astype(np.float32)
    y = rng.standard_normal(geo.m).astype(np.float32)
    return o, f, g, y


@pytest.mark.parametrize("case", edge_cases(), ids=lambda c: c[0])
def test_vjp_one_step_against_oracle(torch, ctis, oracle_mod, case):
    name, geo, ptr, idx, val, box = case
    log(f"vjp one step: {name} geo={geo} box={box}")
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val, box=box, keep_zeros=True)
    o, f, g, y = problem(oracle_mod, geo, ptr, idx, val, 5)
    ws = p.vjp_workspace()
    ws.fill_(float("nan"))                           # scratch contents must not matter
    dv = torch.zeros(p.info.n_entries, device="cuda")
    df = p.em_vjp(torch.from_numpy(g).cuda(), torch.from_numpy(f).cuda(), torch.from_numpy(y).cuda(),
                  dvalues=dv, workspace=ws).cpu().numpy()
    df_o, dv_o = o.em_vjp(g, f, y)
    e_f, e_v = rel_l2(df, df_o), rel_l2(dv.cpu().numpy(), dv_o)
    log(f"  df {e_f:.2e}  dv {e_v:.2e}")
    assert e_f <= DF_TOL
    assert e_v <= DV_TOL


def test_vjp_in_place_accumulate_and_determinism(torch, ctis, oracle_mod):
    c = W.make_case(1)
    p = ctis.Plan.from_case(c, keep_zeros=True)
    geo = c.geometry
    o, f, g, y = problem(oracle_mod, geo, c.lambda_ptr, c.fpa_index, c.value, 8)
    gt, ft, yt = (torch.from_numpy(v).cuda() for v in (g, f, y))
    ws = p.vjp_workspace()
    dv1 = torch.zeros(p.info.n_entries, device="cuda")
    df1 = p.em_vjp(gt, ft, yt, dvalues=dv1, workspace=ws).clone()
    y2 = yt.clone().view(p.shape_f)
    dv2 = torch.full((p.info.n_entries,), 2.0, device="cuda")
    p.em_vjp(gt, ft, y2, df=y2, dvalues=dv2, accumulate=True, workspace=ws)
    assert torch.equal(y2.reshape(-1), df1.reshape(-1)), "in-place df differs"
    assert torch.allclose(dv2 - 2.0, dv1, rtol=0, atol=1e-6 * dv1.abs().max().item())
    dv3 = torch.zeros_like(dv1)
    df3 = p.em_vjp(gt, ft, yt, dvalues=dv3, workspace=ws)
    assert torch.equal(df3, df1) and torch.equal(dv3, dv1), "repeated calls differ"


def test_set_values_matches_a_fresh_plan(torch, ctis):
    c = W.make_case(1)
    geo = c.geometry
    rng = np.random.default_rng(4)
    v2 = (c.value * rng.uniform(0.5, 1.5, c.value.size)).astype(np.float32)
    p1 = ctis.Plan.from_case(c, keep_zeros=True)
    p2 = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, c.lambda_ptr, c.fpa_index, v2, keep_zeros=True)
    p1.set_values(torch.from_numpy(v2).cuda())
    f = torch.rand(p1.shape_f, device="cuda")
    r = torch.rand(p1.shape_g, device="cuda")
    assert torch.equal(p1.forward(f), p2.forward(f))
    assert torch.equal(p1.adjoint(r), p2.adjoint(r))
    g = p2.forward(f) + 0.01
    assert torch.equal(p1.em(g, 3), p2.em(g, 3))


def test_set_values_reaches_every_host_reader(torch, ctis):
    """After set_values, a batch and a Fourier plan built from the plan, its
    column sums, its exported boxes and its sign flag equal those of a plan
    created with the new values (the host copies are re-read from the
    device)."""
    c = W.make_case(1)
    geo = c.geometry
    rng = np.random.default_rng(5)
    v2 = (c.value * rng.uniform(0.5, 1.5, c.value.size)).astype(np.float32)
    p1 = ctis.Plan.from_case(c, keep_zeros=True)
    p2 = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, c.lambda_ptr, c.fpa_index, v2, keep_zeros=True)
    p1.set_values(torch.from_numpy(v2).cuda())
    assert np.array_equal(p1.lambda_sums(), p2.lambda_sums())
    for a, b in zip(p1.boxes(), p2.boxes()):
        assert np.array_equal(a, b)
    f = torch.rand(p1.shape_f, device="cuda")
    g = p2.forward(f) + 0.01
    b1, b2 = ctis.Batch([p1, p1]), ctis.Batch([p2, p2])
    g2 = torch.cat([g.reshape(-1), g.reshape(-1)])
    assert torch.equal(b1.em(g2, 3), b2.em(g2, 3))
    F1, F2 = ctis.Fourier(p1), ctis.Fourier(p2)
    assert torch.equal(F1.forward(f), F2.forward(f))
    assert torch.equal(F1.em(g, 2), F2.em(g, 2))
    # a negative value set on the device reaches the sign flag and the EM check
    v3 = v2.copy()
    v3[0] = -v3[0]
    p1.set_values(torch.from_numpy(v3).cuda())
    assert not p1.info.nonnegative
    with pytest.raises(ctis.CtisError) as ei:
        p1.em(g, 1)
    assert ei.value.name == "CTIS_E_NEGATIVE"
    p1.set_values(torch.from_numpy(v2).cuda())
    assert p1.info.nonnegative
    for x in (F1, F2, b1, b2, p1, p2):
        x.close()


def test_wrong_tensor_arguments_raise_before_any_launch(torch, ctis):
    """Wrong element count, dtype, device or layout raises ValueError in the
    binding; no kernel sees the pointer."""
    c = W.make_case(1)
    p = ctis.Plan.from_case(c)
    b = ctis.Batch([p, p])
    g = torch.rand(p.shape_g, device="cuda")
    f = torch.ones(p.shape_f, device="cuda")
    ws = p.workspace()
    bad = [
        lambda: p.em(g, 1, f=torch.ones(p.sizes.m - 1, device="cuda")),
        lambda: p.em(g, 1, f=torch.ones(p.shape_f, device="cuda", dtype=torch.float64)),
        lambda: p.em(g, 1, f=torch.ones(p.shape_f)),
        lambda: p.em(g, 1, f=f, workspace=torch.empty(4, device="cuda")),
        lambda: p.em_forward_ratio(f[:, :, :-1], g, ws),
        lambda: p.em_adjoint_update(ws, f, torch.empty(p.sizes.m + 1, device="cuda")),
        lambda: p.forward(f, out=torch.empty(p.sizes.n - 1, device="cuda")),
        lambda: b.forward(torch.ones(p.sizes.m, device="cuda")),
        lambda: b.em(torch.cat([g.reshape(-1), g.reshape(-1)])[:-1], 1),
        lambda: b.em(torch.cat([g.reshape(-1), g.reshape(-1)]), 1,
                     f_all=torch.ones(2 * p.sizes.m, device="cuda")[::2].contiguous()[:-1]),
        lambda: b.adjoint(torch.ones(2 * p.sizes.n, device="cuda"), out=torch.empty(3, device="cuda")),
    ]
    for k, fn in enumerate(bad):
        with pytest.raises(ValueError):
            fn()
    assert torch.equal(f, torch.ones_like(f))
    b.close()
    p.close()


def test_value_derivatives_need_the_full_structure(torch, ctis):
    geo = W.Geometry(5, 7, 3, 13, 11)
    ptr, idx, val = W.random_kernels(geo, 9, np.random.default_rng(3))
    first = slice(ptr[0], ptr[1])
    val[first][idx[first] == idx[4]] = 0.0          # every entry at that position: merges to 0
    p = ctis.Plan(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    assert p.info.dropped
    f = torch.rand(p.shape_f, device="cuda")
    g = p.forward(f) + 0.1
    dv = torch.zeros(p.info.n_entries, device="cuda")
    with pytest.raises(ctis.CtisError) as ei:
        p.em_vjp(g, f, f, dvalues=dv)
    assert ei.value.name == "CTIS_E_ARG"
    p.em_vjp(g, f, f)                                 # df alone is fine
    with pytest.raises(ctis.CtisError):
        p.set_values(torch.ones(p.info.n_entries, device="cuda"))


def test_batch_vjp_sums_shared_values(torch, ctis, oracle_mod):
    """Frames 0 and 2 share a plan: the batch's value derivative of that plan
    is the sum of the two frames' derivatives; df is per frame."""
    geos = [W.Geometry(5, 4, 3, 23, 17), W.Geometry(70, 6, 2, 90, 30)]
    rng = np.random.default_rng(9)
    kern = [W.random_kernels(g, 10, rng, clustered=True) for g in geos]
    plans = [ctis.Plan(g.a, g.alpha, g.w, g.gamma, g.xi, *k, box=3, keep_zeros=True) for g, k in zip(geos, kern)]
    order = [0, 1, 0]
    b = ctis.Batch([plans[k] for k in order])
    fo, go = b.f_offsets, b.g_offsets
    orc = [oracle_mod.Oracle(geos[k].a, geos[k].alpha, geos[k].w, geos[k].gamma, geos[k].xi, kern[k][0], kern[k][1],
                             kern[k][2].astype(np.float64)) for k in order]
    f = rng.uniform(0.5, 1.5, fo[-1]).astype(np.float32)
    g = np.concatenate([orc[k].forward(rng.uniform(0.2, 2, geos[order[k]].m)) * rng.uniform(0.7, 1.3, geos[order[k]].n)
                        for k in range(3)]).astype(np.float32)
    y = rng.standard_normal(fo[-1]).astype(np.float32)
    dv = torch.zeros(b.info["n_entries"], device="cuda")
    df = b.em_vjp(torch.from_numpy(g).cuda(), torch.from_numpy(f).cuda(), torch.from_numpy(y).cuda(),
                  dvalues=dv).cpu().numpy()
    dv = dv.cpu().numpy()
    ref = [orc[k].em_vjp(g[go[k]:go[k + 1]], f[fo[k]:fo[k + 1]], y[fo[k]:fo[k + 1]]) for k in range(3)]
    for k in range(3):
        assert rel_l2(df[fo[k]:fo[k + 1]], ref[k][0]) <= DF_TOL
    off0, n0 = b.plan_entries(0)
    off1, n1 = b.plan_entries(1)
    assert (off0, n0) == b.plan_entries(2) and off1 == n0
    assert rel_l2(dv[off0:off0 + n0], ref[0][1] + ref[2][1]) <= DV_TOL
    assert rel_l2(dv[off1:off1 + n1], ref[1][1]) <= DV_TOL


def test_unrolled_gradients_c1_against_oracle(torch, ctis, oracle_mod):
    """16 x 16 x 8 sub-problem (a = alpha = 16, w = 8, FPA 128), K = 10 unrolled
    iterations, loss ||f^(K+1) - f_true||^2: the autograd Function's
    gradients of f0 and of every calibration value against the oracle's
    explicit-H gradient."""
    from paper_2006_01573_amd.autodiff import unrolled_em
    c = W.make_case(1)
    o = oracle_mod.Oracle.from_case(c)
    g = c.noisy(o.forward(c.f_true.ravel()))
    K = 10
    rng = np.random.default_rng(2)
    f0 = rng.uniform(0.5, 1.5, c.geometry.m).astype(np.float32)
    p = ctis.Plan.from_case(c, keep_zeros=True)
    f0_t = torch.tensor(f0, device="cuda", requires_grad=True)
    v_t = torch.tensor(c.value, dtype=torch.float32, device="cuda", requires_grad=True)
    t = torch.tensor(c.f_true.ravel(), dtype=torch.float32, device="cuda")
    fK = unrolled_em(p, torch.from_numpy(g).cuda(), f0_t, K, values=v_t)
    loss = ((fK - t) ** 2).sum()
    loss.backward()
    target = c.f_true.ravel()
    fK_o, df0_o, dv_o = o.unrolled_grad(g, f0.astype(np.float64), K, lambda x: 2.0 * (x - target))
    e_fK = rel_l2(fK.detach().cpu().numpy(), fK_o)
    e_f0, e_v = rel_l2(f0_t.grad.cpu().numpy(), df0_o), rel_l2(v_t.grad.cpu().numpy(), dv_o)
    log(f"c1 K={K}: f {e_fK:.2e} grad f0 {e_f0:.2e} grad values {e_v:.2e}")
    assert e_fK <= GRAD_TOL
    assert e_f0 <= GRAD_TOL
    assert e_v <= GRAD_TOL


@pytest.mark.timeout(600)
def test_c5_gradients_against_finite_differences(torch, ctis, oracle_mod):
    """8 frames of the c2 shape sharing one calibration, K = 10 unrolled
    iterations, loss sum_frames ||f^(K+1) - f_true||^2.  Gradients at 64
    random coordinates (32 of f0, 32 of the calibration values) against
    FP64 central finite differences (h = 1e-6) of the oracle's EM."""
    from paper_2006_01573_amd.autodiff import unrolled_em
    K = 10
    cases = W.differentiable_cases(8, iters=K)
    c0 = cases[0]
    geo = c0.geometry
    o = oracle_mod.Oracle.from_case(c0)
    images = [c.noisy(o.forward(c.f_true.ravel())) for c in cases]
    plan = ctis.Plan.from_case(c0, keep_zeros=True)
    b = ctis.Batch([plan] * len(cases))
    g_all = b.pack_g(images)
    rng = np.random.default_rng(55)
    f0 = rng.uniform(0.5, 1.5, int(b.f_offsets[-1])).astype(np.float32)
    target = np.concatenate([c.f_true.ravel() for c in cases])
    f0_t = torch.tensor(f0, device="cuda", requires_grad=True)
    v_t = torch.tensor(c0.value, dtype=torch.float32, device="cuda", requires_grad=True)
    fK = unrolled_em(b, g_all, f0_t, K, values=v_t)
    loss = ((fK - torch.tensor(target, dtype=torch.float32, device="cuda")) ** 2).sum()
    loss.backward()
    gf0 = f0_t.grad.cpu().numpy()
    gv = v_t.grad.cpu().numpy()
    log(f"c5: GPU gradients done (loss {loss.item():.4e})")

    h = 1e-6
    m = geo.m
    f0d = f0.astype(np.float64)

    def loss_diff(fp, fm, t):
        return ((fp - fm) * (fp + fm - 2 * t)).sum()

    fd_f, gpu_f = [], []
    for j in rng.choice(f0.size, 32, replace=False):
        k = int(j // m)
        sl = slice(k * m, (k + 1) * m)
        e = np.zeros(m)
        e[j - k * m] = h
        fp = o.em(images[k], K, f0=f0d[sl] + e)
        fm = o.em(images[k], K, f0=f0d[sl] - e)
        fd_f.append(loss_diff(fp, fm, target[sl]) / (2 * h))
        gpu_f.append(gf0[j])
    e_f = rel_l2(gpu_f, fd_f)
    log(f"c5: f0 coordinates vs FD rel-L2 {e_f:.2e}")
    fd_v, gpu_v = [], []
    val = c0.value.astype(np.float64)
    for t in rng.choice(val.size, 32, replace=False):
        dv = np.zeros(val.size)
        dv[t] = h
        op = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, c0.lambda_ptr, c0.fpa_index, val + dv)
        om = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, c0.lambda_ptr, c0.fpa_index, val - dv)
        tot = 0.0
        for k in range(len(cases)):
            sl = slice(k * m, (k + 1) * m)
            tot += loss_diff(op.em(images[k], K, f0=f0d[sl]), om.em(images[k], K, f0=f0d[sl]), target[sl])
        fd_v.append(tot / (2 * h))
        gpu_v.append(gv[t])
    e_v = rel_l2(gpu_v, fd_v)
    log(f"c5: value coordinates vs FD rel-L2 {e_v:.2e}")
    assert e_f <= GRAD_TOL
    assert e_v <= GRAD_TOL


def test_vjp_in_a_hip_graph(torch, ctis, oracle_mod):
    """The derivative call allocates and synchronises nothing, so it can be
    captured; replays (with eager work in between) reproduce the eager result."""
    c = W.make_case(1)
    p = ctis.Plan.from_case(c, keep_zeros=True)
    o, f, g, y = problem(oracle_mod, c.geometry, c.lambda_ptr, c.fpa_index, c.value, 12)
    gt, ft, yt = (torch.from_numpy(v).cuda() for v in (g, f, y))
    ws = p.vjp_workspace()
    df = torch.empty(p.shape_f, device="cuda")
    dv = torch.zeros(p.info.n_entries, device="cuda")
    p.em_vjp(gt, ft, yt, df=df, dvalues=dv, workspace=ws)
    ref_df, ref_dv = df.clone(), dv.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        p.em_vjp(gt, ft, yt, df=df, dvalues=dv, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        p.em_vjp(gt, ft, yt, df=df, dvalues=dv, workspace=ws)
    for rep in range(3):
        junk = torch.rand(1 << 20, device="cuda").sum()
        df.zero_()
        dv.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(df, ref_df) and torch.equal(dv, ref_dv), f"replay {rep} differs"
        del junk


def test_unrolled_gradients_on_a_batch_of_distinct_plans(torch, ctis, oracle_mod):
    """The autograd Function over a batch of three frames (two distinct plans,
    one shared): gradients of f0 per frame and of each plan's values (summed
    over the frames that share them) against the oracle; and the f0-only
    path (no values given)."""
    from paper_2006_01573_amd.autodiff import unrolled_em
    geos = [W.Geometry(5, 4, 3, 23, 17), W.Geometry(9, 6, 2, 40, 30)]
    rng = np.random.default_rng(61)
    kern = [W.random_kernels(g, 10, rng, clustered=True) for g in geos]
    plans = [ctis.Plan(g.a, g.alpha, g.w, g.gamma, g.xi, *k, box=3, keep_zeros=True) for g, k in zip(geos, kern)]
    order = [0, 1, 0]
    b = ctis.Batch([plans[k] for k in order])
    orc = [oracle_mod.Oracle(geos[k].a, geos[k].alpha, geos[k].w, geos[k].gamma, geos[k].xi, kern[k][0],
                             kern[k][1], kern[k][2].astype(np.float64)) for k in range(2)]
    fo, go = b.f_offsets, b.g_offsets
    K = 4
    f0 = rng.uniform(0.5, 1.5, fo[-1]).astype(np.float32)
    tgt = rng.uniform(0.2, 2.0, fo[-1])
    g = np.concatenate([orc[order[k]].forward(rng.uniform(0.2, 2, geos[order[k]].m))
                        for k in range(3)]).astype(np.float32)
    vals = np.concatenate([kern[0][2], kern[1][2]]).astype(np.float32)
    f0_t = torch.tensor(f0, device="cuda", requires_grad=True)
    v_t = torch.tensor(vals, device="cuda", requires_grad=True)
    fK = unrolled_em(b, torch.from_numpy(g).cuda(), f0_t, K, values=v_t)
    ((fK - torch.tensor(tgt, dtype=torch.float32, device="cuda")) ** 2).sum().backward()
    gf0, gv = f0_t.grad.cpu().numpy(), v_t.grad.cpu().numpy()
    dv_ref = [np.zeros(kern[0][2].size), np.zeros(kern[1][2].size)]
    for k in range(3):
        sl = slice(fo[k], fo[k + 1])
        t = tgt[sl]
        _, df0, dv = orc[order[k]].unrolled_grad(g[go[k]:go[k + 1]], f0[sl].astype(np.float64), K,
                                                 lambda x, t=t: 2.0 * (x - t))
        assert rel_l2(gf0[sl], df0) <= GRAD_TOL
        dv_ref[order[k]] += dv
    n0 = kern[0][2].size
    assert b.plan_entries(1) == (n0, kern[1][2].size)
    assert rel_l2(gv[:n0], dv_ref[0]) <= GRAD_TOL
    assert rel_l2(gv[n0:], dv_ref[1]) <= GRAD_TOL
    f0_b = torch.tensor(f0, device="cuda", requires_grad=True)
    fK2 = unrolled_em(b, torch.from_numpy(g).cuda(), f0_b, K)
    ((fK2 - torch.tensor(tgt, dtype=torch.float32, device="cuda")) ** 2).sum().backward()
    assert torch.allclose(f0_b.grad, f0_t.grad, rtol=1e-5, atol=1e-6 * f0_t.grad.abs().max().item())
