"""CPU checks of the stored expected values of the large single-frame
workload (tests/golden/c3_expected.npz, written by make_c3_expected.py from
the oracle's assembled H): sampled rows and columns recomputed one by one
from the circulant definition (a separate code path of the oracle that never
assembles H), the frame's photon counts, and the EM flux identity of the
stored iterate."""
import os
import sys

import numpy as np
import pytest

from paper_2006_01573_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "c3_expected.npz")


@pytest.fixture(scope="module")
def stored():
    sys.path.insert(0, os.path.join(HERE, "golden"))
    from make_c3_expected import inputs_sha
    exp = dict(np.load(GOLDEN, allow_pickle=False))
    case = W.make_case(3)
    assert str(exp["inputs_sha"]) == inputs_sha(case)
    return case, exp


def test_stored_projections_match_rows_and_columns(oracle_mod, stored):
    case, exp = stored
    geo = case.geometry
    ok = oracle_mod.Oracle.from_case(case, assemble=False)
    rng = np.random.default_rng(2006)
    f = case.f_true.astype(np.float32).ravel()
    hf = exp["hf"].astype(np.float64)
    rows = np.concatenate([rng.choice(geo.n, 600, replace=False), rng.choice(np.flatnonzero(hf), 600)])
    ref = ok.forward_rows(f, rows)
    assert np.allclose(hf[rows], ref, rtol=1e-6, atol=1e-6 * np.abs(hf).max())
    g = W.frame_from_counts(exp["counts"], float(exp["scale"]))
    cols = rng.choice(geo.m, 600, replace=False)
    ref = ok.adjoint_cols(g, cols)
    htg = exp["htg"].astype(np.float64)
    assert np.allclose(htg[cols], ref, rtol=1e-6, atol=1e-6 * np.abs(htg).max())


def test_stored_frame_and_iterates(oracle_mod, stored):
    case, exp = stored
    geo = case.geometry
    counts = exp["counts"]
    assert counts.dtype == np.uint16 and counts.size == geo.n
    # counts vanish where the clean image does (Poisson(0) = 0); peak 1e4 photons
    assert not np.any(counts[exp["hf"] == 0])
    assert abs(float(exp["scale"]) * float(exp["hf"].astype(np.float64).max()) - 1e4) < 1.0
    for k in ("f100", "f200"):
        assert np.all(np.isfinite(exp[k])) and np.all(exp[k] >= 0)
    # flux identity of EM: sum_j h_j f_j = sum of g over the pixels the
    # projection reaches (here: all pixels with counts), h_s = sum of c_s
    ok = oracle_mod.Oracle.from_case(case, assemble=False)
    cp, _, cv = ok.calibration()
    h = np.repeat(np.add.reduceat(cv, cp[:-1]) if cv.size else np.zeros(geo.w), geo.ell)
    flux = float(np.dot(h, exp["f200"].astype(np.float64)))
    assert abs(flux - float(exp["flux200"])) <= 1e-6 * abs(float(exp["flux200"]))
    assert abs(float(exp["flux200"]) - float(exp["sum_g"])) <= 1e-9 * float(exp["sum_g"])
    # the float32 probe stays well inside the EM tolerance
    assert float(exp["drift200"]) < 1e-4
