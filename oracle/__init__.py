"""FP64 CPU oracle for CTIS EM reconstruction (explicit system matrix).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the product path never does.  It does
not import the HIP package and the HIP package does not import it.

The arithmetic lives in ``ctis_oracle.c`` (plain C, double precision, built
with gcc); this module builds and loads it and converts numpy arrays.
Each function cites the passage of the paper it follows:

  * ``Oracle``       -- H assembled column by column from the shifted
                        calibration images (Sec. 2 calibration + shift
                        invariance; Sec. 3 eq. (decomposition) H_s = C_s E and
                        the zero-based index map).
  * ``forward``      -- g = H f (Sec. 2 eq. (linear)).
  * ``adjoint``      -- z = H^T r (Sec. 3 eq. for H^T u).
  * ``colsums``      -- h_j = sum_i H_ij (Sec. 2, below eq. (em)).
  * ``em``           -- f^(k+1) = (f^(k) . H^T(g / H f^(k))) / h, K times from the
                        given start (Sec. 2 eq. (em); operation order of the
                        Sec. 3 algorithm).
  * ``forward_rows`` / ``adjoint_cols`` -- single rows / columns of H straight
                        from the circulant definition, for sampled checks at
                        sizes where assembling H is too large.
  * ``em_vjp``       -- reverse-mode derivative of one EM step (Sec. 2 eq. (em))
                        with respect to its input f and to the calibration
                        values (the entries of H come from them through
                        Sec. 3's H_s = C_s E), by the chain rule stage by stage.
  * ``unrolled_grad`` -- the same through K unrolled EM steps: the steps run
                        forward keeping every iterate, then their derivatives
                        are applied last to first.
  * ``em_float32_probe`` -- NOT an oracle: the same EM steps in float storage
                        and float accumulation, to estimate how much of a
                        tolerance float rounding alone takes after K steps.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ctis_oracle.c")
_LIB = os.path.join(_HERE, "libctis_oracle.so")
_lock = threading.Lock()
_lib = None

STATUS = {0: "ok", 1: "bad argument", 2: "index out of range", 3: "non-finite value",
          5: "out of memory", 7: "negative calibration value"}


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (strict IEEE double: no fast-math, no FMA
    contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               "-Wno-unused-parameter", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ci = ctypes.c_int
        L.oracle_create.argtypes = [ctypes.POINTER(P), ci, ci, ci, ci, ci, i64p, i32p, f64p, ci]
        L.oracle_create.restype = ci
        L.oracle_create_kernels_only.argtypes = [ctypes.POINTER(P), ci, ci, ci, ci, ci, i64p, i32p, f64p]
        L.oracle_create_kernels_only.restype = ci
        L.oracle_free.argtypes = [P]
        L.oracle_free.restype = None
        L.oracle_nnz.argtypes = [P]
        L.oracle_nnz.restype = ctypes.c_int64
        L.oracle_export_csc.argtypes = [P, i64p, i32p, f64p]
        L.oracle_export_csc.restype = None
        L.oracle_colsums.argtypes = [P, f64p]
        L.oracle_colsums.restype = None
        L.oracle_forward.argtypes = [P, f64p, f64p]
        L.oracle_forward.restype = ci
        L.oracle_adjoint.argtypes = [P, f64p, f64p]
        L.oracle_adjoint.restype = ci
        L.oracle_em.argtypes = [P, f64p, f64p, ci, P]
        L.oracle_em.restype = ci
        L.oracle_smart.argtypes = [P, f64p, f64p, ci]
        L.oracle_smart.restype = ci
        L.oracle_sart.argtypes = [P, f64p, f64p, ci, ctypes.c_double]
        L.oracle_sart.restype = ci
        L.oracle_diagnostics.argtypes = [P, f64p, f64p, f64p,
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
        L.oracle_diagnostics.restype = None
        L.oracle_index_map.argtypes = [P, ctypes.c_int64]
        L.oracle_index_map.restype = ctypes.c_int64
        L.oracle_set_threads.argtypes = [P, ci]
        L.oracle_set_threads.restype = None
        L.oracle_threads_used.argtypes = [P]
        L.oracle_threads_used.restype = ci
        L.oracle_forward_rows.argtypes = [P, f64p, i64p, ctypes.c_int64, f64p]
        L.oracle_forward_rows.restype = None
        L.oracle_adjoint_cols.argtypes = [P, f64p, i64p, ctypes.c_int64, f64p]
        L.oracle_adjoint_cols.restype = None
        L.oracle_cal_nnz.argtypes = [P]
        L.oracle_cal_nnz.restype = ctypes.c_int64
        L.oracle_export_cal.argtypes = [P, i64p, i64p, f64p]
        L.oracle_export_cal.restype = None
        L.oracle_em_vjp.argtypes = [P, f64p, f64p, f64p, f64p, ctypes.c_int64, P, P, P]
        L.oracle_em_vjp.restype = ci
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        L.oracle_em_f32.argtypes = [P, f32p, f32p, ci]
        L.oracle_em_f32.restype = ci
        _lib = L
        return L


def _check(st: int):
    if st != 0:
        raise OracleError(f"oracle: {STATUS.get(st, st)}")


class Oracle:
    """Explicit sparse H in FP64 for one geometry and one set of calibration
    images.  ``assemble=False`` keeps only the calibration vectors (enough for
    ``forward_rows`` / ``adjoint_cols``)."""

    def __init__(self, a, alpha, w, gamma, xi, lambda_ptr, fpa_index, value,
                 assemble: bool = True, threads: int = 0):
        self._L = _load()
        self.a, self.alpha, self.w, self.gamma, self.xi = map(int, (a, alpha, w, gamma, xi))
        self.n = self.gamma * self.xi
        self.ell = self.a * self.alpha
        self.m = self.ell * self.w
        ptr = np.ascontiguousarray(lambda_ptr, dtype=np.int64)
        idx = np.ascontiguousarray(fpa_index, dtype=np.int32)
        val = np.ascontiguousarray(value, dtype=np.float64)
        if ptr.shape != (self.w + 1,):
            raise OracleError("lambda_ptr must have w+1 entries")
        if idx.size < ptr[-1] or val.size < ptr[-1]:
            raise OracleError("fewer calibration entries than lambda_ptr[w]")
        h = ctypes.c_void_p()
        if assemble:
            st = self._L.oracle_create(ctypes.byref(h), self.a, self.alpha, self.w,
                                       self.gamma, self.xi, ptr, idx, val, 1)
        else:
            st = self._L.oracle_create_kernels_only(ctypes.byref(h), self.a, self.alpha,
                                                    self.w, self.gamma, self.xi, ptr, idx, val)
        _check(st)
        self._h = h
        self.assembled = assemble
        self.entries = (ptr.copy(), idx[: ptr[-1]].copy(), val[: ptr[-1]].copy())
        if threads:
            self._L.oracle_set_threads(self._h, int(threads))

    @classmethod
    def from_case(cls, case, **kw):
        g = case.geometry
        return cls(g.a, g.alpha, g.w, g.gamma, g.xi, case.lambda_ptr, case.fpa_index,
                   case.value, **kw)

    def close(self):
        if getattr(self, "_h", None):
            self._L.oracle_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_threads(self, k: int):
        self._L.oracle_set_threads(self._h, int(k))

    @property
    def threads(self) -> int:
        return int(self._L.oracle_threads_used(self._h))

    def _need_h(self):
        if not self.assembled:
            raise OracleError("this oracle was built without the assembled H")

    # -- structure -----------------------------------------------------------
    def index_map(self, j: int) -> int:
        return int(self._L.oracle_index_map(self._h, int(j)))

    def csc(self):
        self._need_h()
        nnz = int(self._L.oracle_nnz(self._h))
        cp = np.empty(self.m + 1, np.int64)
        ri = np.empty(max(nnz, 1), np.int32)
        v = np.empty(max(nnz, 1), np.float64)
        self._L.oracle_export_csc(self._h, cp, ri, v)
        return cp, ri[:nnz], v[:nnz]

    def dense(self) -> np.ndarray:
        """Dense n x m copy of the assembled H (tiny shapes only)."""
        cp, ri, v = self.csc()
        H = np.zeros((self.n, self.m))
        for j in range(self.m):
            for k in range(cp[j], cp[j + 1]):
                H[ri[k], j] += v[k]
        return H

    def calibration(self):
        nnz = int(self._L.oracle_cal_nnz(self._h))
        cp = np.empty(self.w + 1, np.int64)
        ci = np.empty(max(nnz, 1), np.int64)
        cv = np.empty(max(nnz, 1), np.float64)
        self._L.oracle_export_cal(self._h, cp, ci, cv)
        return cp, ci[:nnz], cv[:nnz]

    # -- arithmetic ----------------------------------------------------------
    def colsums(self) -> np.ndarray:
        self._need_h()
        h = np.empty(self.m, np.float64)
        self._L.oracle_colsums(self._h, h)
        return h

    def forward(self, f) -> np.ndarray:
        self._need_h()
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
        if f.size != self.m:
            raise OracleError("f must have m entries")
        g = np.empty(self.n, np.float64)
        _check(self._L.oracle_forward(self._h, f, g))
        return g

    def adjoint(self, r) -> np.ndarray:
        self._need_h()
        r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(-1))
        if r.size != self.n:
            raise OracleError("r must have n entries")
        z = np.empty(self.m, np.float64)
        _check(self._L.oracle_adjoint(self._h, r, z))
        return z

    def em(self, g, iters: int, f0=None, trace: bool = False):
        """K EM iterations from f0 (default all ones).  Returns f^(K+1), and if
        ``trace`` also an array (K, 2) of (flux after the step, loglik before)."""
        self._need_h()
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1))
        if g.size != self.n:
            raise OracleError("g must have n entries")
        f = (np.ones(self.m) if f0 is None
             else np.array(np.asarray(f0, dtype=np.float64).reshape(-1), copy=True))
        if f.size != self.m:
            raise OracleError("f0 must have m entries")
        tr = np.empty(2 * max(iters, 1), np.float64) if trace else None
        st = self._L.oracle_em(self._h, g, f, int(iters),
                               tr.ctypes.data_as(ctypes.c_void_p) if trace else None)
        _check(st)
        if trace:
            return f, tr[: 2 * iters].reshape(iters, 2)
        return f

    def _start(self, g, f0):
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1))
        if g.size != self.n:
            raise OracleError("g must have n entries")
        f = (np.ones(self.m) if f0 is None
             else np.array(np.asarray(f0, dtype=np.float64).reshape(-1), copy=True))
        if f.size != self.m:
            raise OracleError("f0 must have m entries")
        return g, f

    def smart(self, g, iters: int, f0=None) -> np.ndarray:
        """K iterations of simultaneous MART from f0 (default all ones):
        f' = f exp(H^T log(g / H f) / h), log terms 0 where g or H f <= 0."""
        self._need_h()
        g, f = self._start(g, f0)
        _check(self._L.oracle_smart(self._h, g, f, int(iters)))
        return f

    def sart(self, g, iters: int, f0=None, relax: float = 1.0) -> np.ndarray:
        """K iterations of simultaneous ART kept nonnegative, from f0 (default
        all ones): f' = max(0, f + relax H^T((g - H f) / H1) / h)."""
        self._need_h()
        g, f = self._start(g, f0)
        _check(self._L.oracle_sart(self._h, g, f, int(iters), float(relax)))
        return f

    def em_float32_probe(self, g, iters: int, f0=None) -> np.ndarray:
        """The FP32 drift probe (not the oracle): ``iters`` EM iterations with
        float storage and float accumulation in the explicit H's row / column
        order.  Its distance from ``em`` estimates the float rounding floor."""
        self._need_h()
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float32).reshape(-1))
        if g.size != self.n:
            raise OracleError("g must have n entries")
        f = (np.ones(self.m, np.float32) if f0 is None
             else np.array(np.asarray(f0, dtype=np.float32).reshape(-1), copy=True))
        if f.size != self.m:
            raise OracleError("f0 must have m entries")
        _check(self._L.oracle_em_f32(self._h, g, f, int(iters)))
        return f

    def diagnostics(self, g, f):
        """(flux sum_j h_j f_j, Poisson log-likelihood of f)."""
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1))
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
        ghat = self.forward(f)
        fl = ctypes.c_double()
        L = ctypes.c_double()
        self._L.oracle_diagnostics(self._h, g, f, ghat, ctypes.byref(fl), ctypes.byref(L))
        return fl.value, L.value

    def forward_rows(self, f, rows) -> np.ndarray:
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.empty(rows.size, np.float64)
        self._L.oracle_forward_rows(self._h, f, rows, rows.size, out)
        return out

    def adjoint_cols(self, r, cols) -> np.ndarray:
        r = np.ascontiguousarray(np.asarray(r, dtype=np.float64).reshape(-1))
        cols = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.empty(cols.size, np.float64)
        self._L.oracle_adjoint_cols(self._h, r, cols, cols.size, out)
        return out

    # -- derivatives ---------------------------------------------------------
    def em_vjp(self, g, f, y, positions=None):
        """One EM step's reverse-mode derivative at input ``f`` for the upstream
        gradient ``y`` = dL/df'.  Returns (dL/df, dL/dv) where dL/dv holds, for
        every calibration entry given at construction (in that order; entries
        that share a position get the same value), the derivative with respect
        to that entry's value.  ``positions`` = (lambda, index) arrays picks
        other calibration positions instead."""
        self._need_h()
        g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1))
        f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape(-1))
        y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(-1))
        if g.size != self.n or f.size != self.m or y.size != self.m:
            raise OracleError("g must have n entries, f and y m entries")
        if positions is None:
            ptr, idx, _ = self.entries
            lam = np.repeat(np.arange(self.w, dtype=np.int32), np.diff(ptr))
            pos = idx.astype(np.int64)
        else:
            lam = np.ascontiguousarray(positions[0], dtype=np.int32)
            pos = np.ascontiguousarray(positions[1], dtype=np.int64)
        df = np.empty(self.m, np.float64)
        dv = np.empty(max(lam.size, 1), np.float64)
        st = self._L.oracle_em_vjp(self._h, g, f, y, df, lam.size,
                                   lam.ctypes.data_as(ctypes.c_void_p),
                                   pos.ctypes.data_as(ctypes.c_void_p),
                                   dv.ctypes.data_as(ctypes.c_void_p))
        _check(st)
        return df, dv[: lam.size]

    def unrolled_grad(self, g, f0, iters: int, dL_df):
        """Derivatives of a loss of f^(K+1) (K = ``iters`` EM steps from f0)
        with respect to f0 and to the calibration entries' values, given
        ``dL_df`` -- a function of f^(K+1) returning dL/df^(K+1).  Returns
        (f^(K+1), dL/df0, dL/dv)."""
        f = np.array(np.asarray(f0, dtype=np.float64).reshape(-1), copy=True)
        iterates = [f.copy()]
        for _ in range(iters):
            f = self.em(g, 1, f0=f)
            iterates.append(f.copy())
        y = np.asarray(dL_df(f), dtype=np.float64).reshape(-1)
        dv = np.zeros(int(self.entries[0][-1]), np.float64)
        for k in range(iters - 1, -1, -1):
            y, dvk = self.em_vjp(g, iterates[k], y)
            dv += dvk
        return f, y, dv
