"""Pins for the oracle's simultaneous MART (SMART) and simultaneous ART
(SART, kept nonnegative): the other solvers Sec. 2 names beside EM (cited
there to Gordon, Bender and Herman), in the simultaneous form that applies
every ray's correction at once through H and H^T.

Each test ties the oracle to something fixed independently of its code:
  * closed forms: a single voxel (H is one column c: SMART reaches the
    c-weighted geometric mean of g_i / c_i in one step, SART with relaxation
    lam moves the fraction lam of the way to sum g / sum c), and the delta
    calibration (H = E: SMART reaches E^T g in one step, SART moves the
    fraction lam of the way to it);
  * fixed points for noiseless data;
  * scaling laws (SMART: g -> t g scales the iterates by t, the calibration
    -> t c scales them by 1/t; SART: (g, f0) -> t (g, f0) scales them by t);
  * a dense implementation on tiny inputs whose H is built from the paper's
    literal matrices (Sec. 3: H_s = C_s E), not from the oracle's assembly.
"""
import numpy as np
import pytest
import scipy.linalg

from paper_2006_01573_amd import workloads as W


def literal_H(geo, ptr, idx, val):
    c = np.zeros((geo.w, geo.n))
    for s in range(geo.w):
        np.add.at(c[s], idx[ptr[s]:ptr[s + 1]].astype(np.int64), val[ptr[s]:ptr[s + 1]].astype(np.float64))
    Q = np.vstack([np.eye(geo.a), np.zeros((geo.gamma - geo.a, geo.a))])
    top = np.kron(np.eye(geo.alpha), Q)
    E = np.vstack([top, np.zeros((geo.n - top.shape[0], geo.ell))])
    return np.hstack([scipy.linalg.circulant(c[s]) @ E for s in range(geo.w)])


def make_oracle(oracle_mod, geo, ptr, idx, val):
    return oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val)


def single_voxel(oracle_mod, seed):
    geo = W.Geometry(1, 1, 1, 5, 3)
    rng = np.random.default_rng(seed)
    c = rng.random(geo.n) + 0.05
    c[[2, 7]] = 0.0
    nz = np.flatnonzero(c)
    o = make_oracle(oracle_mod, geo, np.array([0, nz.size], np.int64), nz.astype(np.int32), c[nz])
    g = rng.random(geo.n) * 3 + 0.1
    return o, c, g


def test_smart_single_voxel_closed_form(oracle_mod):
    o, c, g = single_voxel(oracle_mod, 4)
    on = c > 0
    expected = np.exp((c[on] * np.log(g[on] / c[on])).sum() / c.sum())
    for f0 in (1.0, 0.3, 17.0):
        np.testing.assert_allclose(o.smart(g, 1, f0=np.array([f0])), [expected], rtol=1e-13)
        np.testing.assert_allclose(o.smart(g, 4, f0=np.array([f0])), [expected], rtol=1e-13)


@pytest.mark.parametrize("lam", [1.0, 0.5, 1.5])
def test_sart_single_voxel_closed_form(oracle_mod, lam):
    o, c, g = single_voxel(oracle_mod, 5)
    target = g[c > 0].sum() / c.sum()
    for f0 in (1.0, 0.3, 17.0):
        expected = max(0.0, (1 - lam) * f0 + lam * target)
        np.testing.assert_allclose(o.sart(g, 1, f0=np.array([f0]), relax=lam), [expected], rtol=1e-13)


def delta_oracle(oracle_mod):
    geo = W.Geometry(4, 3, 1, 6, 5)
    o = make_oracle(oracle_mod, geo, np.array([0, 1], np.int64), np.zeros(1, np.int32), np.ones(1, np.float32))
    return geo, o


def test_smart_delta_one_step_is_crop(oracle_mod):
    geo, o = delta_oracle(oracle_mod)
    rng = np.random.default_rng(8)
    g = rng.random((geo.xi, geo.gamma)) + 0.05
    f0 = rng.random(geo.m) + 0.1
    np.testing.assert_allclose(o.smart(g.ravel(), 1, f0=f0), g[:geo.alpha, :geo.a].ravel(), rtol=1e-13)


@pytest.mark.parametrize("lam", [1.0, 0.25])
def test_sart_delta_step_moves_towards_crop(oracle_mod, lam):
    geo, o = delta_oracle(oracle_mod)
    rng = np.random.default_rng(9)
    g = rng.random((geo.xi, geo.gamma))
    f0 = rng.random(geo.m) + 0.1
    crop = g[:geo.alpha, :geo.a].ravel()
    np.testing.assert_allclose(o.sart(g.ravel(), 1, f0=f0, relax=lam), (1 - lam) * f0 + lam * crop, rtol=1e-13)


@pytest.mark.parametrize("solver", ["smart", "sart"])
def test_fixed_point_noiseless(oracle_mod, solver):
    case = W.make_case(1)
    o = oracle_mod.Oracle.from_case(case)
    f_true = case.f_true.astype(np.float64).ravel() + 0.01   # strictly positive
    g = o.forward(f_true)
    f = getattr(o, solver)(g, 5, f0=f_true)
    np.testing.assert_allclose(f, f_true, rtol=1e-11)


GEOS = [W.Geometry(3, 2, 2, 5, 4), W.Geometry(2, 3, 3, 6, 5), W.Geometry(4, 4, 2, 7, 6)]


def tiny(geo, seed):
    rng = np.random.default_rng([11, seed])
    ptr, idx, val = W.random_kernels(geo, 5, rng)
    idx[0] = geo.n - 1                       # an image that wraps round the FPA's end
    return ptr, idx, val, rng


@pytest.mark.parametrize("gi", range(len(GEOS)))
def test_smart_scaling_laws(oracle_mod, gi):
    geo = GEOS[gi]
    ptr, idx, val, rng = tiny(geo, gi)
    o = make_oracle(oracle_mod, geo, ptr, idx, val)
    o_t = make_oracle(oracle_mod, geo, ptr, idx, val.astype(np.float64) * 2.5)
    g = rng.random(geo.n) + 0.1              # positive everywhere: every log term counts
    for k in (1, 3):
        f = o.smart(g, k)
        np.testing.assert_allclose(o.smart(3.0 * g, k), 3.0 * f, rtol=1e-12)
        np.testing.assert_allclose(o_t.smart(g, k), f / 2.5, rtol=1e-12)


@pytest.mark.parametrize("gi", range(len(GEOS)))
def test_sart_homogeneity(oracle_mod, gi):
    geo = GEOS[gi]
    ptr, idx, val, rng = tiny(geo, 10 + gi)
    o = make_oracle(oracle_mod, geo, ptr, idx, val)
    g = rng.random(geo.n)
    f0 = rng.random(geo.m) + 0.1
    for k in (1, 3):
        np.testing.assert_allclose(o.sart(4.0 * g, k, f0=4.0 * f0, relax=0.7), 4.0 * o.sart(g, k, f0=f0, relax=0.7),
                                   rtol=1e-12)


@pytest.mark.parametrize("gi", range(len(GEOS)))
def test_dense_literal_matrices(oracle_mod, gi):
    """Both solvers against loops over a dense H made from the literal C_s and
    E (wrapping images included), with zeros in g to exercise the zero rules."""
    geo = GEOS[gi]
    ptr, idx, val, rng = tiny(geo, 20 + gi)
    o = make_oracle(oracle_mod, geo, ptr, idx, val)
    H = literal_H(geo, ptr, idx, val)
    h = H.sum(0)
    R = H.sum(1)
    g = rng.random(geo.n) + 0.05
    g[rng.random(geo.n) < 0.2] = 0.0
    f_s = np.ones(geo.m)
    f_a = np.ones(geo.m)
    for _ in range(3):
        gh = H @ f_s
        ok = (g > 0) & (gh > 0)
        l = np.zeros(geo.n)
        l[ok] = np.log(g[ok] / gh[ok])
        f_s = np.where(h != 0, f_s * np.exp((H.T @ l) / np.where(h != 0, h, 1)), 0.0)
        gh = H @ f_a
        r = np.where(R != 0, (g - gh) / np.where(R != 0, R, 1), 0.0)
        f_a = np.where(h != 0, np.maximum(0.0, f_a + 0.8 * (H.T @ r) / np.where(h != 0, h, 1)), 0.0)
    np.testing.assert_allclose(o.smart(g, 3), f_s, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(o.sart(g, 3, relax=0.8), f_a, rtol=1e-12, atol=1e-14)


def test_smart_refuses_negative_calibration(oracle_mod):
    geo = GEOS[0]
    ptr, idx, val, _ = tiny(geo, 30)
    val = val.copy()
    val[0] = -0.5
    o = make_oracle(oracle_mod, geo, ptr, idx, val)
    with pytest.raises(oracle_mod.OracleError):
        o.smart(np.ones(geo.n), 1)
