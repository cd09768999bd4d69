"""Pins for the oracle's derivatives of EM (one step and K unrolled steps).

The oracle differentiates the EM step of Sec. 2 eq. (em) stage by stage.  Each
test below ties that to something fixed independently of its code:

  * central finite differences of the oracle's own EM iteration (whose
    arithmetic is pinned in test_oracle_pins.py), along random directions in
    f and in the calibration values, and coordinate by coordinate;
  * torch's reverse-mode autodiff of a dense float64 EM written from the
    paper's literal matrices (C_s circulant from c_s, E = [I_alpha (x) Q; 0]);
  * closed forms of the step: f' is homogeneous of degree 0 in f and of
    degree -1 in the calibration values (Euler's relation then fixes
    <f, dL/df> and <v, dL/dv>), and with the upstream gradient y = h the
    step's weighted flux sum_j h_j f'_j equals sum_i g_i on the support, so
    dL/df vanishes and dL/dv reduces to the column-sum term.
"""
import numpy as np
import pytest

from paper_2006_01573_amd import workloads as W

GEOS = [W.Geometry(4, 3, 3, 11, 9), W.Geometry(5, 4, 2, 23, 17), W.Geometry(3, 3, 4, 13, 11)]


def make_problem(oracle_mod, geo, seed, nnz=6, clustered=True):
    rng = np.random.default_rng(seed)
    ptr, idx, val = W.random_kernels(geo, nnz, rng, clustered=clustered)
    val = val.astype(np.float64)
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    f_true = rng.uniform(0.2, 2.0, geo.m)
    g = o.forward(f_true) * rng.uniform(0.7, 1.3, geo.n)
    f = rng.uniform(0.5, 1.5, geo.m)
    return rng, (ptr, idx, val), o, f, g


def step(oracle_mod, geo, cal, f, g):
    ptr, idx, val = cal
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    return o.em(g, 1, f0=f)


@pytest.mark.parametrize("geo", GEOS, ids=str)
def test_vjp_matches_directional_finite_differences(oracle_mod, geo):
    rng, cal, o, f, g = make_problem(oracle_mod, geo, 11)
    y = rng.standard_normal(geo.m)
    df, dv = o.em_vjp(g, f, y)
    h = 1e-6
    # along f
    d = rng.standard_normal(geo.m)
    fd = y @ (o.em(g, 1, f0=f + h * d) - o.em(g, 1, f0=f - h * d)) / (2 * h)
    assert abs(fd - df @ d) <= 1e-7 * (abs(fd) + np.abs(df).sum() * 1e-3 + 1e-12)
    # along the calibration values
    ptr, idx, val = cal
    dval = rng.standard_normal(val.size)
    fp = step(oracle_mod, geo, (ptr, idx, val + h * dval), f, g)
    fm = step(oracle_mod, geo, (ptr, idx, val - h * dval), f, g)
    fd_v = y @ (fp - fm) / (2 * h)
    assert abs(fd_v - dv @ dval) <= 1e-6 * (abs(fd_v) + 1e-9)


def test_vjp_matches_finite_differences_per_coordinate(oracle_mod):
    geo = GEOS[0]
    rng, cal, o, f, g = make_problem(oracle_mod, geo, 5, nnz=5)
    y = rng.standard_normal(geo.m)
    df, dv = o.em_vjp(g, f, y)
    h = 1e-6
    for j in range(geo.m):
        e = np.zeros(geo.m)
        e[j] = h
        fd = y @ (o.em(g, 1, f0=f + e) - o.em(g, 1, f0=f - e)) / (2 * h)
        assert fd == pytest.approx(df[j], rel=1e-6, abs=1e-8 * np.abs(df).max())
    ptr, idx, val = cal
    for t in range(val.size):
        e = np.zeros(val.size)
        e[t] = h
        fd = y @ (step(oracle_mod, geo, (ptr, idx, val + e), f, g)
                  - step(oracle_mod, geo, (ptr, idx, val - e), f, g)) / (2 * h)
        assert fd == pytest.approx(dv[t], rel=1e-6, abs=1e-8 * np.abs(dv).max())


def dense_torch_em_grad(geo, cal, f0, g, iters, target):
    """Reverse-mode autodiff (torch, float64) of K EM steps built from the
    paper's literal matrices: C_s[i, q] = c_s[(i - q) mod n], H_s = C_s E."""
    import torch
    ptr, idx, val = cal
    lam = np.repeat(np.arange(geo.w), np.diff(ptr))
    v = torch.tensor(val, dtype=torch.float64, requires_grad=True)
    f = torch.tensor(f0, dtype=torch.float64, requires_grad=True)
    c = torch.zeros(geo.w, geo.n, dtype=torch.float64).index_put(
        (torch.as_tensor(lam), torch.as_tensor(idx.astype(np.int64))), v, accumulate=True)
    ii = np.arange(geo.n)
    shift = torch.as_tensor((ii[:, None] - ii[None, :]) % geo.n)
    Q = np.vstack([np.eye(geo.a), np.zeros((geo.gamma - geo.a, geo.a))])
    top = np.kron(np.eye(geo.alpha), Q)
    E = torch.tensor(np.vstack([top, np.zeros((geo.n - top.shape[0], geo.ell))]))
    H = torch.cat([c[s][shift] @ E for s in range(geo.w)], dim=1)
    gt = torch.tensor(g)
    h = H.sum(0)
    x = f
    for _ in range(iters):
        ghat = H @ x
        pos = ghat > 0
        u = torch.where(pos, gt / torch.where(pos, ghat, torch.ones_like(ghat)), torch.zeros_like(ghat))
        zeta = H.T @ u
        nz = h != 0
        x = torch.where(nz, x * zeta / torch.where(nz, h, torch.ones_like(h)), torch.zeros_like(h))
    loss = ((x - torch.tensor(target)) ** 2).sum()
    loss.backward()
    return x.detach().numpy(), f.grad.numpy(), v.grad.numpy()


@pytest.mark.parametrize("geo", GEOS[:2], ids=str)
def test_unrolled_grad_matches_dense_autodiff(oracle_mod, geo):
    rng, cal, o, f, g = make_problem(oracle_mod, geo, 23)
    target = rng.uniform(0.2, 2.0, geo.m)
    K = 4
    fK, df0, dv = o.unrolled_grad(g, f, K, lambda x: 2.0 * (x - target))
    fK_t, df0_t, dv_t = dense_torch_em_grad(geo, cal, f, g, K, target)
    np.testing.assert_allclose(fK, fK_t, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(df0, df0_t, rtol=1e-9, atol=1e-12 * np.abs(df0_t).max())
    np.testing.assert_allclose(dv, dv_t, rtol=1e-9, atol=1e-12 * np.abs(dv_t).max())


def test_unrolled_grad_matches_finite_differences(oracle_mod):
    geo = GEOS[1]
    rng, cal, o, f, g = make_problem(oracle_mod, geo, 31)
    target = rng.uniform(0.2, 2.0, geo.m)
    K = 5
    _, df0, dv = o.unrolled_grad(g, f, K, lambda x: 2.0 * (x - target))

    def loss_diff(fp, fm):
        # L(+) - L(-) evaluated term by term: sum (fp - fm)(fp + fm - 2t)
        return ((fp - fm) * (fp + fm - 2 * target)).sum()

    h = 1e-6
    # rounding of the iterates (~1e-16 relative each) summed over the m terms
    # of the loss difference, divided by 2h: ~1e-9 absolute noise in each FD
    noise = 50 * np.finfo(float).eps * np.sqrt(geo.m) * 4.0 / (2 * h)
    for j in rng.choice(geo.m, 8, replace=False):
        e = np.zeros(geo.m)
        e[j] = h
        fd = loss_diff(o.em(g, K, f0=f + e), o.em(g, K, f0=f - e)) / (2 * h)
        assert fd == pytest.approx(df0[j], rel=1e-6, abs=noise)
    ptr, idx, val = cal
    for t in rng.choice(val.size, 8, replace=False):
        e = np.zeros(val.size)
        e[t] = h
        op = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val + e)
        om = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val - e)
        fd = loss_diff(op.em(g, K, f0=f), om.em(g, K, f0=f)) / (2 * h)
        assert fd == pytest.approx(dv[t], rel=1e-6, abs=noise)


@pytest.mark.parametrize("geo", GEOS, ids=str)
def test_vjp_euler_relations(oracle_mod, geo):
    """f'(c f) = f'(f) and f'(f; c v) = f'(f; v) / c, so by Euler's relation
    <f, dL/df> = 0 and <v, dL/dv> = -<y, f'>."""
    rng, cal, o, f, g = make_problem(oracle_mod, geo, 41)
    y = rng.standard_normal(geo.m)
    df, dv = o.em_vjp(g, f, y)
    f1 = o.em(g, 1, f0=f)
    scale = np.abs(df * f).sum()
    assert abs(df @ f) <= 1e-12 * scale
    assert cal[2] @ dv == pytest.approx(-(y @ f1), rel=1e-11)


@pytest.mark.parametrize("geo", GEOS, ids=str)
def test_vjp_with_column_sum_weights(oracle_mod, geo):
    """With y = h the loss sum_j h_j f'_j equals sum of g over pixels with
    H f > 0, which does not move with f: dL/df = 0; and dL/dv_t reduces to the
    column-sum term -sum_{j in s} f'_j of the entry's wavelength s."""
    rng, cal, o, f, g = make_problem(oracle_mod, geo, 53)
    h = o.colsums()
    df, dv = o.em_vjp(g, f, h)
    assert np.abs(df).max() <= 1e-12 * np.abs(h * o.adjoint(np.ones(geo.n))).max()
    f1 = o.em(g, 1, f0=f).reshape(geo.w, geo.ell)
    ptr = cal[0]
    expect = np.repeat(-f1.sum(axis=1), np.diff(ptr))
    np.testing.assert_allclose(dv, expect, rtol=1e-10, atol=1e-12 * np.abs(expect).max())


def test_vjp_zero_wavelength_and_dead_pixels(oracle_mod):
    """A wavelength whose values are all zero has h_s = 0 and f'_s = 0 for any
    input, so dL/df_s = 0; pixels with H f = 0 contribute nothing."""
    geo = W.Geometry(4, 3, 3, 11, 9)
    rng = np.random.default_rng(3)
    ptr, idx, val = W.random_kernels(geo, 4, rng, clustered=True)
    val = val.astype(np.float64)
    val[ptr[1]:ptr[2]] = 0.0
    o = oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)
    f = rng.uniform(0.5, 1.5, geo.m)
    g = o.forward(f) * 1.1
    y = rng.standard_normal(geo.m)
    df, dv = o.em_vjp(g, f, y)
    assert np.all(df[geo.ell:2 * geo.ell] == 0.0)
    assert np.all(np.isfinite(dv))
    # the loss does not depend on f_s for that wavelength: FD agrees (zero)
    e = np.zeros(geo.m)
    e[geo.ell + 3] = 1e-6
    assert y @ (o.em(g, 1, f0=f + e) - o.em(g, 1, f0=f - e)) == 0.0


def test_vjp_rejects_bad_positions(oracle_mod):
    geo = GEOS[0]
    rng, cal, o, f, g = make_problem(oracle_mod, geo, 2)
    with pytest.raises(oracle_mod.OracleError):
        o.em_vjp(g, f, f, positions=(np.array([geo.w]), np.array([0])))
    with pytest.raises(oracle_mod.OracleError):
        o.em_vjp(g, f, f, positions=(np.array([0]), np.array([geo.n])))
