"""Seeded synthetic CTIS workloads.

This module only draws inputs: sensor geometry, sparse per-wavelength
calibration images, a ground-truth datacube and Poisson noise for a clean FPA
image that the caller computes.  It holds none of the reconstruction's
arithmetic (no projection, no EM step), so the oracle side and the HIP side can
both take their inputs from here.

Layout conventions (the paper's column-major vectorisation, Sec. 3 index map):
  * datacube f: numpy array of shape (w, alpha, a); voxel (x, y, s) sits at
    flat index j = x + a*y + a*alpha*s.
  * FPA image g: shape (xi, gamma); pixel (r, c) sits at flat index
    i = r + gamma*c.
  * calibration image of wavelength s: COO entries (fpa_index, value) in
    lambda_ptr[s] .. lambda_ptr[s+1], fpa_index = r + gamma*c.  It is the image
    of a point source at field-stop pixel (0, 0) (Sec. 2: each calibration
    image becomes the first column of its wavelength block of H).

Synthetic model (the paper's measured calibration and scene are not
available, so these stand in for them):
  * diffraction orders (p, q) in {-P..P}^2; order (p, q) of wavelength s is
    centred at (r0 + p*d_s, c0 + q*d_s) with (r0, c0) = ((gamma-a)//2,
    (xi-alpha)//2), so the zeroth-order image of the whole field stop is
    centred on the FPA;
  * each order is a (2R+1)^2 Gaussian blob, peak-normalised: value
    A*exp(-(dr^2+dc^2)/(2 sigma^2)); zeroth-order amplitude 1, first orders
    U(0.5, 1), second orders U(0.1, 0.3);
  * f_true[s, y, x] = M(x, y) * S_xy(s), with S a sum of 3 Gaussians in the
    wavelength index and M a sum of 4 spatial Gaussian blobs.
"""
from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np

SEED_ROOT = 200601573


@dataclasses.dataclass(frozen=True)
class Geometry:
    a: int          # field-stop extent along the FPA's fast axis (gamma)
    alpha: int      # field-stop extent along the slow axis (xi)
    w: int          # number of wavelengths
    gamma: int      # FPA fast-axis extent
    xi: int         # FPA slow-axis extent

    @property
    def n(self) -> int:
        return self.gamma * self.xi

    @property
    def ell(self) -> int:
        return self.a * self.alpha

    @property
    def m(self) -> int:
        return self.ell * self.w


@dataclasses.dataclass(frozen=True)
class KernelModel:
    orders: int                          # P: orders (p, q) with |p|, |q| <= P
    radius: int                          # R: blob is (2R+1) x (2R+1)
    sigma: float
    dispersion: Callable[[int], int]     # d_s in pixels for wavelength index s


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    geometry: Geometry
    kernel: KernelModel
    iters: int
    noise: str          # "scale" (fixed photon scale) or "peak" (peak photons)
    photons: float


def _d_c1(s: int) -> int:
    return 20 + 2 * s


def _d_c2(s: int) -> int:
    return 80 + 3 * s


def _d_c3(s: int) -> int:
    return 60 + 2 * s


def _d_256(s: int) -> int:
    return 40 + 2 * s


CONFIGS = {
    1: Config("c1-small a=alpha=16 w=8 FPA128",
              Geometry(16, 16, 8, 128, 128), KernelModel(1, 1, 0.8, _d_c1),
              iters=20, noise="scale", photons=1e3),
    2: Config("c2-paper-shaped a=alpha=64 w=32 FPA512",
              Geometry(64, 64, 32, 512, 512), KernelModel(1, 1, 0.8, _d_c2),
              iters=100, noise="peak", photons=1e4),
    3: Config("c3-large a=alpha=128 w=64 FPA1024",
              Geometry(128, 128, 64, 1024, 1024), KernelModel(2, 2, 1.2, _d_c3),
              iters=200, noise="peak", photons=1e4),
}


def rng_for(cfg: int, frame: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, cfg, frame]))


def order_amplitude(rng: np.random.Generator, p: int, q: int) -> float:
    k = max(abs(p), abs(q))
    if k == 0:
        return 1.0
    if k == 1:
        return float(rng.uniform(0.5, 1.0))
    return float(rng.uniform(0.1, 0.3))


def make_kernels(geo: Geometry, km: KernelModel, rng: np.random.Generator):
    """Sparse calibration images, one per wavelength, as COO.

    Returns (lambda_ptr int64[w+1], fpa_index int32[nnz], value float32[nnz]).
    Entries of one wavelength are in the order orders-row-major, then blob
    row-major; no duplicates are produced.
    """
    r0 = (geo.gamma - geo.a) // 2
    c0 = (geo.xi - geo.alpha) // 2
    R = km.radius
    dr, dc = np.meshgrid(np.arange(-R, R + 1), np.arange(-R, R + 1), indexing="ij")
    dr = dr.ravel()
    dc = dc.ravel()
    shape = np.exp(-(dr.astype(np.float64) ** 2 + dc.astype(np.float64) ** 2)
                   / (2.0 * km.sigma ** 2))
    ptr = [0]
    idx_all = []
    val_all = []
    for s in range(geo.w):
        d = km.dispersion(s)
        for p in range(-km.orders, km.orders + 1):
            for q in range(-km.orders, km.orders + 1):
                amp = order_amplitude(rng, p, q)
                rr = r0 + p * d + dr
                cc = c0 + q * d + dc
                if rr.min() < 0 or rr.max() >= geo.gamma or cc.min() < 0 or cc.max() >= geo.xi:
                    raise ValueError("diffraction order falls off the FPA")
                idx_all.append((rr + geo.gamma * cc).astype(np.int64))
                val_all.append(amp * shape)
        ptr.append(ptr[-1] + (2 * km.orders + 1) ** 2 * dr.size)
    idx = np.concatenate(idx_all).astype(np.int32)
    val = np.concatenate(val_all).astype(np.float32)
    return np.asarray(ptr, dtype=np.int64), idx, val


def make_ftrue(geo: Geometry, rng: np.random.Generator) -> np.ndarray:
    """Nonnegative smooth datacube, shape (w, alpha, a), float64."""
    w, a, al = geo.w, geo.a, geo.alpha
    lam = np.arange(w, dtype=np.float64)
    # per-pixel spectra: 3 Gaussians in the wavelength index
    A = rng.uniform(0.2, 1.0, size=(al, a, 3))
    mu = rng.uniform(0.0, max(w - 1, 0), size=(al, a, 3))
    sw = rng.uniform(w / 16.0, w / 4.0, size=(al, a, 3))
    spec = np.zeros((w, al, a))
    for k in range(3):
        spec += A[None, :, :, k] * np.exp(
            -((lam[:, None, None] - mu[None, :, :, k]) ** 2) / (2.0 * sw[None, :, :, k] ** 2))
    # spatial mask: 4 Gaussian blobs
    cx = rng.uniform(0.0, a, size=4)
    cy = rng.uniform(0.0, al, size=4)
    rho = rng.uniform(a / 16.0, a / 4.0, size=4)
    x = np.arange(a, dtype=np.float64)[None, :]
    y = np.arange(al, dtype=np.float64)[:, None]
    mask = np.zeros((al, a))
    for b in range(4):
        mask += np.exp(-((x - cx[b]) ** 2 + (y - cy[b]) ** 2) / (2.0 * rho[b] ** 2))
    return spec * mask[None, :, :]


def noise_counts(clean: np.ndarray, mode: str, photons: float,
                 rng: np.random.Generator):
    """Poisson photon counts on a clean FPA image and their scale.

    mode "scale": counts = Poisson(photons * clean), s = photons.
    mode "peak":  s = photons / max(clean); counts = Poisson(s * clean).
    Returns (counts int64, s); the frame is ``frame_from_counts(counts, s)``.
    """
    clean = np.asarray(clean, dtype=np.float64)
    if np.any(clean < 0):
        raise ValueError("clean image must be nonnegative")
    if mode == "scale":
        s = float(photons)
    elif mode == "peak":
        peak = float(clean.max())
        s = photons / peak if peak > 0 else 1.0
    else:
        raise ValueError(mode)
    return rng.poisson(s * clean), s


def frame_from_counts(counts: np.ndarray, s: float) -> np.ndarray:
    """g = counts / s, float32."""
    return (np.asarray(counts, dtype=np.float64) / s).astype(np.float32)


def add_noise(clean: np.ndarray, mode: str, photons: float,
              rng: np.random.Generator) -> np.ndarray:
    """Poisson noise on a clean FPA image: g = Poisson(s * clean) / s (float32),
    s as in ``noise_counts``."""
    counts, s = noise_counts(clean, mode, photons, rng)
    return frame_from_counts(counts, s)


@dataclasses.dataclass
class Case:
    """One synthetic frame: geometry, kernels, ground truth and a noise stream.

    The clean image H f_true is not computed here; the caller forms it and
    passes it to ``noisy``.
    """
    cfg: Config
    lambda_ptr: np.ndarray
    fpa_index: np.ndarray
    value: np.ndarray
    f_true: np.ndarray          # float64 (w, alpha, a)
    rng: np.random.Generator    # continues after the kernel and f_true draws

    @property
    def geometry(self) -> Geometry:
        return self.cfg.geometry

    def noisy(self, clean: np.ndarray) -> np.ndarray:
        return add_noise(clean, self.cfg.noise, self.cfg.photons, self.rng)


def make_case(cfg_id: int, frame: int = 0, cfg: Config | None = None) -> Case:
    cfg = cfg if cfg is not None else CONFIGS[cfg_id]
    rng = rng_for(cfg_id, frame)
    ptr, idx, val = make_kernels(cfg.geometry, cfg.kernel, rng)
    ft = make_ftrue(cfg.geometry, rng)
    return Case(cfg, ptr, idx, val, ft, rng)


# ---------------------------------------------------------------------------
# batched frames of uneven shapes (one plan and one frame per entry)

def batched_configs(n_frames: int = 64, cfg_id: int = 4):
    """Per-frame configs for the uneven batch: a = alpha in {32, 48, 64},
    w in {16, 32}; FPA 256 when a = 32, else 512; 50 EM iterations."""
    rng = rng_for(cfg_id, 10_000)
    out = []
    for k in range(n_frames):
        a = int(rng.choice([32, 48, 64]))
        w = int(rng.choice([16, 32]))
        fpa = 256 if a == 32 else 512
        d = _d_256 if fpa == 256 else _d_c2
        out.append(Config(f"c4-frame{k} a={a} w={w} FPA{fpa}",
                          Geometry(a, a, w, fpa, fpa), KernelModel(1, 1, 0.8, d),
                          iters=50, noise="peak", photons=1e4))
    return out


# ---------------------------------------------------------------------------
# differentiable unrolled EM: frames of the c2 shape sharing one calibration

def differentiable_cases(n_frames: int = 8, iters: int = 10, cfg_id: int = 5):
    """Frames for the differentiable reconstruction: a = alpha = 64, w = 32,
    FPA 512 (the c2 shape and kernel model), ``iters`` unrolled EM
    iterations, Poisson noise at 1e4 peak photons.  All frames share the
    calibration of frame 0 (one plan); each has its own f_true and noise."""
    base = CONFIGS[2]
    cfg = Config(f"c5-differentiable {n_frames} frames a=alpha=64 w=32 FPA512 K={iters}",
                 base.geometry, base.kernel, iters=iters, noise=base.noise, photons=base.photons)
    ptr, idx, val = make_kernels(cfg.geometry, cfg.kernel, rng_for(cfg_id, 0))
    cases = []
    for k in range(n_frames):
        rng = rng_for(cfg_id, k + 1)
        cases.append(Case(cfg, ptr, idx, val, make_ftrue(cfg.geometry, rng), rng))
    return cases


def random_kernels(geo: Geometry, nnz_per_lambda: int, rng: np.random.Generator,
                   nonneg: bool = True, clustered: bool = False):
    """Arbitrary sparse calibration images (for edge-case tests): uniform random
    positions anywhere on the FPA, including rows and columns at the FPA edges
    so that shifted images wrap.  Duplicated positions are allowed."""
    ptr = [0]
    idx = []
    val = []
    for _ in range(geo.w):
        if clustered:
            cr = rng.integers(0, geo.gamma)
            cc = rng.integers(0, geo.xi)
            rr = (cr + rng.integers(-2, 3, size=nnz_per_lambda)) % geo.gamma
            ccs = (cc + rng.integers(-2, 3, size=nnz_per_lambda)) % geo.xi
            ii = rr + geo.gamma * ccs
        else:
            ii = rng.integers(0, geo.n, size=nnz_per_lambda)
        vv = rng.uniform(0.05, 1.0, size=nnz_per_lambda)
        if not nonneg:
            vv = vv * rng.choice([-1.0, 1.0], size=nnz_per_lambda)
        idx.append(ii)
        val.append(vv)
        ptr.append(ptr[-1] + nnz_per_lambda)
    return (np.asarray(ptr, dtype=np.int64), np.concatenate(idx).astype(np.int32),
            np.concatenate(val).astype(np.float32))
