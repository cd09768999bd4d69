"""Write the expected values of the large single-frame workload (a = alpha =
128, w = 64, 1024 x 1024 FPA, 5 x 5 diffraction orders of 5 x 5 blobs, 200 EM
iterations) from the FP64 oracle alone.

    python tests/golden/make_c3_expected.py [--threads T]

The explicit H of this workload has 655 M nonzeros (about 16 GB as CSC plus
CSR), too large to assemble inside a GPU test; this script assembles it once
on the host and stores, in ``c3_expected.npz``:

  counts, scale   the frame: Poisson photon counts on the oracle's H f_true
                  (f_true rounded to float32, the values the GPU is given) at
                  1e4 peak photons; g = counts / scale as float32
                  (``workloads.frame_from_counts``)
  hf              the oracle's H f_true                      (float32 of FP64)
  htg             the oracle's H^T g                         (float32 of FP64)
  f100, f200      the oracle's EM iterate after 100 and 200 iterations from
                  all ones (Sec. 2 eq. (em), Sec. 3 algorithm) (float32 of FP64)
  flux200, loglik200, sum_g
                  flux sum_j h_j f_j and Poisson log-likelihood
                  sum_i (g_i log ghat_i - ghat_i) of f200, and sum_i g_i
  drift100, drift200
                  relative L2 distance of the FP32 drift probe (float storage
                  and accumulation, not the oracle) from the FP64 EM iterate
  inputs_sha      SHA-256 of the seeded calibration and f_true, so that a
                  changed generator is detected instead of compared against

Nothing here touches the HIP library: only ``oracle`` and the seeded input
generators of ``paper_2006_01573_amd.workloads`` (which hold none of the
method's arithmetic).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "c3_expected.npz")


def inputs_sha(case) -> str:
    h = hashlib.sha256()
    for arr in (case.lambda_ptr, case.fpa_index, case.value, case.f_true.astype(np.float32)):
        h.update(np.ascontiguousarray(arr).tobytes())
    return h.hexdigest()


def rel_l2(x, ref) -> float:
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def main() -> int:
    import oracle
    from paper_2006_01573_amd import workloads as W

    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()

    def log(msg):
        print(f"[c3 golden] {msg}", flush=True)

    case = W.make_case(3)
    geo = case.geometry
    t0 = time.perf_counter()
    log(f"assembling the explicit H ({geo})")
    o = oracle.Oracle.from_case(case, threads=args.threads)
    log(f"assembled in {time.perf_counter() - t0:.1f} s, {o.threads} threads")
    f_true = case.f_true.astype(np.float32).ravel()
    hf = o.forward(f_true)
    counts, scale = W.noise_counts(hf, case.cfg.noise, case.cfg.photons, case.rng)
    if counts.max() > np.iinfo(np.uint16).max:
        raise SystemExit("photon counts do not fit 16 bits")
    g = W.frame_from_counts(counts, scale)
    htg = o.adjoint(g)
    log("projections done; 100 EM iterations")
    t1 = time.perf_counter()
    f100 = o.em(g, 100)
    log(f"100 iterations in {time.perf_counter() - t1:.1f} s; 100 more")
    f200 = o.em(g, 100, f0=f100)
    flux, loglik = o.diagnostics(g, f200)
    log("FP32 drift probe")
    p100 = o.em_float32_probe(g, 100)
    p200 = o.em_float32_probe(g, 100, f0=p100)
    drift100, drift200 = rel_l2(p100, f100), rel_l2(p200, f200)
    log(f"drift of float32 arithmetic: {drift100:.3e} at K=100, {drift200:.3e} at K=200")
    meta = {"workload": case.cfg.name, "iters": [100, 200], "threads": o.threads,
            "seconds": round(time.perf_counter() - t0, 1)}
    np.savez_compressed(
        OUT, counts=counts.astype(np.uint16), scale=np.float64(scale),
        hf=hf.astype(np.float32), htg=htg.astype(np.float32),
        f100=f100.astype(np.float32), f200=f200.astype(np.float32),
        flux200=np.float64(flux), loglik200=np.float64(loglik), sum_g=np.float64(g.astype(np.float64).sum()),
        drift100=np.float64(drift100), drift200=np.float64(drift200),
        inputs_sha=np.array(inputs_sha(case)), meta=np.array(json.dumps(meta)))
    log(f"wrote {OUT} ({os.path.getsize(OUT) / 2**20:.1f} MiB)")
    return 0


if __name__ == "__main__":
    sys.exit(main())
