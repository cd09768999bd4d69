"""Pins for the FP64 oracle: each test ties an oracle function to something
the paper or the mathematics fixes independently of the oracle's own code.

  * hand-worked tiny matrices (tests/golden/hand_worked.json);
  * the paper's literal matrices (Sec. 3: C_s circulant with first column c_s,
    Q = [I_a; 0], E = [I_alpha (x) Q; 0], H_s = C_s E) built with scipy /
    numpy Kronecker products -- a construction different from the oracle's
    column-by-column shifting;
  * the paper's zero-based index maps (Sec. 3) against the literal E;
  * the Fourier route of Sec. 3 (forward eq. with d_s = F c_s, adjoint via the
    Hermitian half spectrum), computed with numpy's rfft / irfft;
  * the adjoint identity <Hf, r> = <f, H^T r>;
  * closed forms: delta calibration (H = I_w (x) E), single voxel EM,
    column sums of a circulant, scaling laws of EM;
  * EM invariants: fixed point, nonnegativity, flux conservation and the
    monotone Poisson likelihood of Shepp & Vardi's EM (cited in Sec. 2);
  * brute-force dense EM on tiny inputs.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg

from paper_2006_01573_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")


# --------------------------------------------------------------------------
# literal constructions from Sec. 3 (independent of the oracle's code)

def literal_c(geo, ptr, idx, val):
    c = np.zeros((geo.w, geo.n))
    for s in range(geo.w):
        np.add.at(c[s], idx[ptr[s]:ptr[s + 1]].astype(np.int64),
                  val[ptr[s]:ptr[s + 1]].astype(np.float64))
    return c


def literal_E(geo):
    Q = np.vstack([np.eye(geo.a), np.zeros((geo.gamma - geo.a, geo.a))])
    top = np.kron(np.eye(geo.alpha), Q)
    return np.vstack([top, np.zeros((geo.n - top.shape[0], geo.ell))])


def literal_H(geo, ptr, idx, val):
    c = literal_c(geo, ptr, idx, val)
    E = literal_E(geo)
    return np.hstack([scipy.linalg.circulant(c[s]) @ E for s in range(geo.w)])


def paper_index_map(geo, j):
    """Sec. 3: i = j - s*ell + (gamma - a) floor((j - s*ell)/a) + s*n, s = floor(j/ell)."""
    s = j // geo.ell
    jp = j - s * geo.ell
    return jp + (geo.gamma - geo.a) * (jp // geo.a) + s * geo.n


def make_oracle(oracle_mod, geo, ptr, idx, val, **kw):
    return oracle_mod.Oracle(geo.a, geo.alpha, geo.w, geo.gamma, geo.xi, ptr, idx, val, **kw)


TINY = [
    W.Geometry(3, 2, 2, 5, 4),      # odd gamma, a < gamma, alpha < xi
    W.Geometry(4, 3, 3, 4, 5),      # a == gamma (no zero rows inside a column block)
    W.Geometry(2, 5, 1, 7, 5),      # alpha == xi
    W.Geometry(1, 1, 2, 3, 3),      # single-pixel field stop
    W.Geometry(5, 4, 2, 6, 7),
]


def tiny_kernels(geo, seed, nnz=6, nonneg=True):
    rng = np.random.default_rng([7, seed])
    ptr, idx, val = W.random_kernels(geo, nnz, rng, nonneg=nonneg)
    # force wrap: entries in the last FPA row and the last pixel
    idx[0] = geo.n - 1
    if idx.size > 1:
        idx[1] = geo.gamma - 1
    # force a duplicate in the first wavelength
    if ptr[1] - ptr[0] >= 3:
        idx[2] = idx[1]
    return ptr, idx, val


# --------------------------------------------------------------------------

def test_hand_worked_examples(oracle_mod):
    with open(GOLDEN) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        o = oracle_mod.Oracle(c["a"], c["alpha"], c["w"], c["gamma"], c["xi"],
                              np.array(c["lambda_ptr"]), np.array(c["fpa_index"]),
                              np.array(c["value"]))
        np.testing.assert_array_equal(o.dense(), np.array(c["H"], float), err_msg=c["name"])
        np.testing.assert_array_equal(o.colsums(), np.array(c["h"], float), err_msg=c["name"])
        np.testing.assert_allclose(o.forward(np.array(c["f"], float)), c["Hf"], rtol=0, atol=1e-15)
        if "em_g" in c:
            f2 = o.em(np.array(c["em_g"], float), 1)
            np.testing.assert_allclose(f2, c["em_f_after_1_from_ones"], rtol=1e-15)


@pytest.mark.parametrize("gi", range(len(TINY)))
@pytest.mark.parametrize("seed", [0, 1])
def test_assembly_equals_literal_matrices(oracle_mod, gi, seed):
    geo = TINY[gi]
    ptr, idx, val = tiny_kernels(geo, seed, nonneg=(seed == 0))
    o = make_oracle(oracle_mod, geo, ptr, idx, val)
    H = literal_H(geo, ptr, idx, val)
    np.testing.assert_array_equal(o.dense(), H)
    # column sums of the literal matrix (signed calibrations when seed == 1)
    np.testing.assert_allclose(o.colsums(), H.sum(0), rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("gi", range(len(TINY)))
def test_index_maps_match_literal_E(oracle_mod, gi):
    geo = TINY[gi]
    E = literal_E(geo)
    IE = np.kron(np.eye(geo.w), E)        # (I_w (x) E), nw x m
    ptr, idx, val = tiny_kernels(geo, 3)
    o = make_oracle(oracle_mod, geo, ptr, idx, val)
    for j in range(geo.m):
        i = paper_index_map(geo, j)
        col = IE[:, j]
        assert col[i] == 1.0 and col.sum() == 1.0            # forward map v_i = f_j
        s = j // geo.ell
        assert o.index_map(j) + s * geo.n == i
        x, y = (j - s * geo.ell) % geo.a, (j - s * geo.ell) // geo.a
        assert i == x + geo.gamma * y + s * geo.n
    # transposed map: zeta = (I_w (x) E)^T z picks z at the same index
    z = np.random.default_rng(5).standard_normal(geo.n * geo.w)
    zeta = IE.T @ z
    for j in range(geo.m):
        assert zeta[j] == z[paper_index_map(geo, j)]


def fft_forward(geo, c, f):
    """Sec. 3 forward eq.: g = F^-1 sum_s d_s . F v_s, d_s = F c_s, v_s = E f_s,
    with the Hermitian half spectrum (length floor(n/2)+1)."""
    E = literal_E(geo)
    acc = np.zeros(geo.n // 2 + 1, complex)
    for s in range(geo.w):
        v = E @ f[s * geo.ell:(s + 1) * geo.ell]
        acc += np.fft.rfft(c[s]) * np.fft.rfft(v)
    return np.fft.irfft(acc, geo.n)


def fft_adjoint(geo, c, u):
    """Sec. 3 back projection: C_s^T u = F^-1 (conj(d_s) . F u), then the
    transposed index map (crop)."""
    E = literal_E(geo)
    U = np.fft.rfft(u)
    out = []
    for s in range(geo.w):
        z = np.fft.irfft(np.conj(np.fft.rfft(c[s])) * U, geo.n)
        out.append(E.T @ z)
    return np.concatenate(out)


@pytest.mark.parametrize("gi", range(len(TINY)))
def test_fourier_route(oracle_mod, gi):
    geo = TINY[gi]
    ptr, idx, val = tiny_kernels(geo, 11, nonneg=False)
    o = make_oracle(oracle_mod, geo, ptr, idx, val)
    c = literal_c(geo, ptr, idx, val)
    rng = np.random.default_rng(12)
    f = rng.standard_normal(geo.m)
    u = rng.standard_normal(geo.n)
    g_ref = fft_forward(geo, c, f)
    z_ref = fft_adjoint(geo, c, u)
    np.testing.assert_allclose(o.forward(f), g_ref, rtol=0, atol=1e-12 * np.abs(g_ref).max())
    np.testing.assert_allclose(o.adjoint(u), z_ref, rtol=0, atol=1e-12 * np.abs(z_ref).max())


def test_fourier_route_c1(oracle_mod):
    case = W.make_case(1)
    geo = case.geometry
    o = oracle_mod.Oracle.from_case(case)
    c = literal_c(geo, case.lambda_ptr, case.fpa_index, case.value)
    rng = np.random.default_rng(13)
    f = rng.random(geo.m)
    u = rng.random(geo.n)

    def Ev(fs):  # literal E is too big to form densely here; index map instead
        v = np.zeros(geo.n)
        j = np.arange(geo.ell)
        v[j % geo.a + geo.gamma * (j // geo.a)] = fs
        return v

    acc = np.zeros(geo.n // 2 + 1, complex)
    for s in range(geo.w):
        acc += np.fft.rfft(c[s]) * np.fft.rfft(Ev(f[s * geo.ell:(s + 1) * geo.ell]))
    g_ref = np.fft.irfft(acc, geo.n)
    np.testing.assert_allclose(o.forward(f), g_ref, rtol=0, atol=1e-12 * g_ref.max())
    U = np.fft.rfft(u)
    j = np.arange(geo.ell)
    z_ref = np.concatenate([
        np.fft.irfft(np.conj(np.fft.rfft(c[s])) * U, geo.n)[j % geo.a + geo.gamma * (j // geo.a)]
        for s in range(geo.w)])
    np.testing.assert_allclose(o.adjoint(u), z_ref, rtol=0, atol=1e-12 * z_ref.max())


@pytest.mark.parametrize("gi", range(len(TINY)))
def test_adjoint_identity(oracle_mod, gi):
    geo = TINY[gi]
    ptr, idx, val = tiny_kernels(geo, 21, nonneg=False)
    o = make_oracle(oracle_mod, geo, ptr, idx, val)
    rng = np.random.default_rng(22)
    for _ in range(3):
        f = rng.standard_normal(geo.m)
        r = rng.standard_normal(geo.n)
        lhs = o.forward(f) @ r
        rhs = f @ o.adjoint(r)
        assert abs(lhs - rhs) <= 1e-13 * (np.abs(o.forward(f)) @ np.abs(r) + 1)


def test_delta_calibration(oracle_mod):
    """c_s = delta at index 0 for every s: H = (I_w (x) E) stacked side by side,
    so H f = sum_s E f_s (zero-padding embed) and H^T r = crop of r per block."""
    geo = W.Geometry(3, 4, 3, 7, 6)
    ptr = np.arange(geo.w + 1, dtype=np.int64)
    idx = np.zeros(geo.w, np.int32)
    val = np.ones(geo.w, np.float32)
    o = make_oracle(oracle_mod, geo, ptr, idx, val)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((geo.w, geo.alpha, geo.a))
    img = np.zeros((geo.xi, geo.gamma))
    img[:geo.alpha, :geo.a] = f.sum(0)
    np.testing.assert_allclose(o.forward(f.ravel()), img.ravel(), rtol=1e-15, atol=1e-15)
    r = rng.standard_normal((geo.xi, geo.gamma))
    crop = np.broadcast_to(r[:geo.alpha, :geo.a], (geo.w, geo.alpha, geo.a))
    np.testing.assert_array_equal(o.adjoint(r.ravel()), crop.ravel())


def test_column_sums_are_kernel_sums(oracle_mod):
    case = W.make_case(1)
    o = oracle_mod.Oracle.from_case(case)
    h = o.colsums().reshape(case.geometry.w, -1)
    p = case.lambda_ptr
    for s in range(case.geometry.w):
        hs = case.value[p[s]:p[s + 1]].astype(np.float64).sum()
        np.testing.assert_allclose(h[s], hs, rtol=1e-14)


def test_single_voxel_closed_form(oracle_mod):
    """a = alpha = w = 1: H is the column c, so one EM step gives
    f = sum_{i: c_i > 0} g_i / sum_i c_i from any positive start."""
    geo = W.Geometry(1, 1, 1, 5, 3)
    rng = np.random.default_rng(4)
    c = rng.random(geo.n)
    c[[2, 7]] = 0.0
    nz = np.flatnonzero(c)
    ptr = np.array([0, nz.size], np.int64)
    o = make_oracle(oracle_mod, geo, ptr, nz.astype(np.int32), c[nz])
    g = rng.random(geo.n) * 3
    expected = g[c > 0].sum() / c.sum()
    for f0 in (1.0, 0.3, 17.0):
        f = o.em(g, 1, f0=np.array([f0]))
        np.testing.assert_allclose(f, [expected], rtol=1e-14)
        np.testing.assert_allclose(o.em(g, 5, f0=np.array([f0])), [expected], rtol=1e-14)


def test_delta_em_one_step_is_crop(oracle_mod):
    """w = 1, c = delta: H = E; one EM step from any positive start gives E^T g."""
    geo = W.Geometry(4, 3, 1, 6, 5)
    o = make_oracle(oracle_mod, geo, np.array([0, 1], np.int64), np.zeros(1, np.int32),
                    np.ones(1, np.float32))
    rng = np.random.default_rng(8)
    g = rng.random((geo.xi, geo.gamma))
    f0 = rng.random(geo.m) + 0.1
    f = o.em(g.ravel(), 1, f0=f0)
    np.testing.assert_allclose(f, g[:geo.alpha, :geo.a].ravel(), rtol=1e-14)


def test_em_scaling_laws(oracle_mod):
    """From f^(1) = 1: scaling g by t scales f^(k) (k >= 2) by t; scaling the
    calibration by t scales f^(k) by 1/t."""
    geo = TINY[0]
    ptr, idx, val = tiny_kernels(geo, 31)
    o = make_oracle(oracle_mod, geo, ptr, idx, val)
    t = 3.5
    o_t = make_oracle(oracle_mod, geo, ptr, idx, val.astype(np.float64) * t)
    g = np.random.default_rng(9).random(geo.n)
    for k in (1, 4):
        f = o.em(g, k)
        np.testing.assert_allclose(o.em(t * g, k), t * f, rtol=1e-13)
        np.testing.assert_allclose(o_t.em(g, k), f / t, rtol=1e-13)


@pytest.fixture(scope="module")
def c1_problem(oracle_mod):
    case = W.make_case(1)
    o = oracle_mod.Oracle.from_case(case)
    clean = o.forward(case.f_true.ravel())
    g = case.noisy(clean)
    return case, o, clean, g


def test_fixed_point_noiseless(c1_problem):
    """Noiseless g = H f_true: f_true is a fixed point of the EM map."""
    case, o, clean, _ = c1_problem
    ft = case.f_true.ravel() + 1e-3       # strictly positive
    g = o.forward(ft)
    f = o.em(g, 10, f0=ft)
    np.testing.assert_allclose(f, ft, rtol=1e-12)


def test_em_invariants_c1(c1_problem):
    case, o, clean, g = c1_problem
    K = case.cfg.iters
    f, tr = o.em(g, K, trace=True)
    assert np.all(f >= 0)
    ghat0 = o.forward(np.ones(o.m))
    # flux: sum_j h_j f_j^(k+1) = sum_{i: ghat_i > 0} g_i  (every iteration)
    target = g.astype(np.float64)[ghat0 > 0].sum()
    np.testing.assert_allclose(tr[:, 0], target, rtol=1e-13)
    np.testing.assert_allclose(target, g.astype(np.float64).sum(), rtol=1e-15)
    # monotone Poisson log-likelihood (Shepp & Vardi)
    L = tr[:, 1]
    assert np.all(np.diff(L) >= -1e-12 * np.abs(L[1:]))
    _, L_end = o.diagnostics(g, f)
    assert L_end >= L[-1] - 1e-12 * abs(L[-1])


@pytest.mark.parametrize("gi", [0, 1, 4])
def test_bruteforce_dense_em(oracle_mod, gi):
    """Dense EM with the literal H (numpy) against the sparse C oracle."""
    geo = TINY[gi]
    ptr, idx, val = tiny_kernels(geo, 41)
    o = make_oracle(oracle_mod, geo, ptr, idx, val)
    H = literal_H(geo, ptr, idx, val)
    h = H.sum(0)
    rng = np.random.default_rng(42)
    g = rng.random(geo.n) * (H.sum(1) > 0)
    f = np.ones(geo.m)
    for _ in range(7):
        gh = H @ f
        u = np.where(gh > 0, g / np.where(gh > 0, gh, 1.0), 0.0)
        f = np.where(h != 0, f * (H.T @ u) / np.where(h != 0, h, 1.0), 0.0)
    np.testing.assert_allclose(o.em(g, 7), f, rtol=1e-13, atol=1e-300)


def test_sampled_rows_and_columns_match_assembly(oracle_mod):
    """forward_rows / adjoint_cols (definition, no assembly) equal the
    assembled H on every row and column, including wrap cases."""
    for gi, geo in enumerate(TINY):
        ptr, idx, val = tiny_kernels(geo, 50 + gi, nonneg=False)
        o = make_oracle(oracle_mod, geo, ptr, idx, val)
        ok = make_oracle(oracle_mod, geo, ptr, idx, val, assemble=False)
        H = literal_H(geo, ptr, idx, val)
        rng = np.random.default_rng(51)
        f = rng.standard_normal(geo.m)
        r = rng.standard_normal(geo.n)
        np.testing.assert_allclose(ok.forward_rows(f, np.arange(geo.n)), H @ f, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(ok.adjoint_cols(r, np.arange(geo.m)), H.T @ r, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(o.forward(f), H @ f, rtol=1e-13, atol=1e-13)


def test_oracle_rejects_bad_input(oracle_mod):
    geo = TINY[0]
    ptr, idx, val = tiny_kernels(geo, 60)
    bad = idx.copy()
    bad[0] = geo.n
    with pytest.raises(oracle_mod.OracleError):
        make_oracle(oracle_mod, geo, ptr, bad, val)
    badv = val.astype(np.float64)
    badv[1] = np.nan
    with pytest.raises(oracle_mod.OracleError):
        make_oracle(oracle_mod, geo, ptr, idx, badv)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.Oracle(5, 2, 1, 4, 4, np.array([0, 1]), np.zeros(1, np.int32), np.ones(1))
    neg = val.astype(np.float64)
    neg[0] = -1.0
    o = make_oracle(oracle_mod, geo, ptr, idx, neg)
    with pytest.raises(oracle_mod.OracleError):
        o.em(np.ones(geo.n), 1)
