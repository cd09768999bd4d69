"""ctypes binding of libctis (the C ABI in include/ctis.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream (``torch.cuda.current_stream()``); every arithmetic step runs in the
library's HIP kernels.  There is no fallback: if libctis.so is missing or the
GPU is absent, the calls raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libctis.so")

CTIS_PLAN_HOST_ONLY = 0x1
CTIS_PLAN_KEEP_ZEROS = 0x2
CTIS_PLAN_TILE_PATH = 0x4
# region shapes of the region EM path (pixels along gamma, xi), by CTIS_PLAN_REGION code
REGION_SHAPES = [None, (8, 32), (16, 16), (32, 8), (16, 8), (8, 16), (8, 8)]
CTIS_BATCH_PERSISTENT = 0x400
CTIS_BATCH_TILE_PATH = 0x8000
CTIS_BATCH_REGION_SOLO = 0x10000
SOLVERS = {"em": 0, "smart": 1, "sart": 2}   # ctis_solver

STATUS_NAMES = {0: "CTIS_OK", 1: "CTIS_E_ARG", 2: "CTIS_E_INDEX", 3: "CTIS_E_VALUE",
                4: "CTIS_E_TOO_LARGE", 5: "CTIS_E_NOMEM", 6: "CTIS_E_HIP",
                7: "CTIS_E_NEGATIVE", 8: "CTIS_E_WORKSPACE"}

# every function include/ctis.h declares
EXPORTED = ["ctis_plan_create", "ctis_plan_destroy", "ctis_plan_get_info",
            "ctis_plan_lambda_sums", "ctis_plan_export_boxes", "ctis_plan_export_worklist",
            "ctis_plan_export_regions", "ctis_em_diagnostics", "ctis_em_iterate_static",
            "ctis_forward", "ctis_adjoint", "ctis_em_iterate", "ctis_em_forward_ratio", "ctis_em_adjoint_update", "ctis_status_str",
            "ctis_last_error", "ctis_version", "ctis_batch_create", "ctis_batch_destroy",
            "ctis_batch_get_info", "ctis_batch_forward", "ctis_batch_adjoint", "ctis_batch_em_iterate",
            "ctis_batch_em_forward_ratio", "ctis_batch_em_adjoint_update", "ctis_solve_iterate",
            "ctis_batch_solve_iterate", "ctis_em_vjp", "ctis_plan_set_values", "ctis_batch_em_vjp", "ctis_batch_set_values",
            "ctis_batch_plan_entries", "ctis_fourier_create", "ctis_fourier_destroy", "ctis_fourier_get_info",
            "ctis_fourier_forward", "ctis_fourier_adjoint", "ctis_fourier_em_iterate"]


def CTIS_PLAN_BOX(b: int) -> int:
    return (int(b) & 0xF) << 8


class CtisError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {detail}")


class _Info(ctypes.Structure):
    _fields_ = [("a", ctypes.c_int32), ("alpha", ctypes.c_int32), ("w", ctypes.c_int32),
                ("gamma", ctypes.c_int32), ("xi", ctypes.c_int32),
                ("n", ctypes.c_int64), ("ell", ctypes.c_int64), ("m", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("n_support", ctypes.c_int64),
                ("box", ctypes.c_int32), ("n_boxes", ctypes.c_int32),
                ("tile_fast", ctypes.c_int32), ("tile_slow", ctypes.c_int32),
                ("n_tiles", ctypes.c_int32), ("n_active_tiles", ctypes.c_int32),
                ("n_items", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t),
                ("nonnegative", ctypes.c_int32), ("device", ctypes.c_int32),
                ("waves_forward", ctypes.c_int32), ("waves_adjoint", ctypes.c_int32),
                ("n_entries", ctypes.c_int64), ("vjp_workspace_bytes", ctypes.c_size_t),
                ("dropped", ctypes.c_int32),
                ("region_fast", ctypes.c_int32), ("region_slow", ctypes.c_int32),
                ("n_regions", ctypes.c_int32), ("n_active_regions", ctypes.c_int32),
                ("n_region_items", ctypes.c_int64), ("em_region_path", ctypes.c_int32),
                ("waves_region", ctypes.c_int32), ("method_madds", ctypes.c_int64),
                ("tile_forward_madds", ctypes.c_int64), ("region_forward_madds", ctypes.c_int64),
                ("adjoint_madds", ctypes.c_int64), ("solve_workspace_bytes", ctypes.c_size_t)]


class _BatchInfo(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("box", ctypes.c_int32),
                ("m_total", ctypes.c_int64), ("n_total", ctypes.c_int64),
                ("forward_units", ctypes.c_int64), ("adjoint_units", ctypes.c_int64),
                ("waves_forward", ctypes.c_int32), ("waves_adjoint", ctypes.c_int32),
                ("workspace_bytes", ctypes.c_size_t), ("n_plans", ctypes.c_int32),
                ("n_entries", ctypes.c_int64), ("vjp_workspace_bytes", ctypes.c_size_t),
                ("em_region_path", ctypes.c_int32), ("waves_region", ctypes.c_int32),
                ("region_units", ctypes.c_int64), ("solve_workspace_bytes", ctypes.c_size_t)]


class _FourierInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n1", ctypes.c_int32), ("n2", ctypes.c_int32),
                ("pairs", ctypes.c_int32), ("spectra_bytes", ctypes.c_size_t),
                ("workspace_bytes", ctypes.c_size_t)]


@dataclasses.dataclass(frozen=True)
class PlanInfo:
    a: int
    alpha: int
    w: int
    gamma: int
    xi: int
    n: int
    ell: int
    m: int
    nnz: int
    n_support: int
    box: int
    n_boxes: int
    tile_fast: int
    tile_slow: int
    n_tiles: int
    n_active_tiles: int
    n_items: int
    workspace_bytes: int
    nonnegative: bool
    device: int
    waves_forward: int
    waves_adjoint: int
    n_entries: int
    vjp_workspace_bytes: int
    dropped: bool
    region_fast: int
    region_slow: int
    n_regions: int
    n_active_regions: int
    n_region_items: int
    em_region_path: bool
    waves_region: int
    method_madds: int
    tile_forward_madds: int
    region_forward_madds: int
    adjoint_madds: int
    solve_workspace_bytes: int


_lock = threading.Lock()
_lib = None


def load_library(path: str | None = None):
    """Load libctis.so (built by ``paper_2006_01573_amd.build``)."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or os.environ.get("CTIS_LIBRARY") or LIB_PATH
        if not os.path.exists(p):
            raise ImportError(f"{p} is missing: build it with `python -m paper_2006_01573_amd.build`")
        L = ctypes.CDLL(p)
        vp = ctypes.c_void_p
        i32, i64, u32, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
        st = ctypes.c_int
        L.ctis_plan_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32, i32, vp, vp, vp, u32]
        L.ctis_plan_create.restype = st
        L.ctis_plan_destroy.argtypes = [vp]
        L.ctis_plan_destroy.restype = None
        L.ctis_plan_get_info.argtypes = [vp, ctypes.POINTER(_Info)]
        L.ctis_plan_get_info.restype = st
        L.ctis_plan_lambda_sums.argtypes = [vp, vp]
        L.ctis_plan_lambda_sums.restype = st
        L.ctis_plan_export_boxes.argtypes = [vp, vp, vp, vp]
        L.ctis_plan_export_boxes.restype = st
        L.ctis_plan_export_worklist.argtypes = [vp, vp, vp]
        L.ctis_plan_export_worklist.restype = st
        L.ctis_plan_export_regions.argtypes = [vp, vp, vp]
        L.ctis_plan_export_regions.restype = st
        L.ctis_forward.argtypes = [vp, vp, vp, vp]
        L.ctis_forward.restype = st
        L.ctis_adjoint.argtypes = [vp, vp, vp, vp]
        L.ctis_adjoint.restype = st
        L.ctis_em_iterate.argtypes = [vp, vp, vp, i32, vp, sz, vp]
        L.ctis_em_iterate.restype = st
        L.ctis_em_iterate_static.argtypes = [vp, vp, vp, i32, vp]
        L.ctis_em_iterate_static.restype = st
        L.ctis_em_diagnostics.argtypes = [vp, vp, vp, vp, vp, sz, vp]
        L.ctis_em_diagnostics.restype = st
        L.ctis_em_forward_ratio.argtypes = [vp, vp, vp, vp, sz, vp]
        L.ctis_em_forward_ratio.restype = st
        L.ctis_em_adjoint_update.argtypes = [vp, vp, sz, vp, vp, vp]
        L.ctis_em_adjoint_update.restype = st
        L.ctis_batch_create.argtypes = [ctypes.POINTER(vp), vp, i32, u32]
        L.ctis_batch_create.restype = st
        L.ctis_batch_destroy.argtypes = [vp]
        L.ctis_batch_destroy.restype = None
        L.ctis_batch_get_info.argtypes = [vp, ctypes.POINTER(_BatchInfo)]
        L.ctis_batch_get_info.restype = st
        L.ctis_batch_forward.argtypes = [vp, vp, vp, vp]
        L.ctis_batch_forward.restype = st
        L.ctis_batch_adjoint.argtypes = [vp, vp, vp, vp]
        L.ctis_batch_adjoint.restype = st
        L.ctis_batch_em_iterate.argtypes = [vp, vp, vp, i32, vp, sz, vp]
        L.ctis_batch_em_iterate.restype = st
        L.ctis_batch_em_forward_ratio.argtypes = [vp, vp, vp, vp, sz, vp]
        L.ctis_batch_em_forward_ratio.restype = st
        L.ctis_batch_em_adjoint_update.argtypes = [vp, vp, sz, vp, vp, vp]
        L.ctis_batch_em_adjoint_update.restype = st
        L.ctis_solve_iterate.argtypes = [vp, i32, vp, vp, i32, ctypes.c_float, vp, sz, vp]
        L.ctis_solve_iterate.restype = st
        L.ctis_batch_solve_iterate.argtypes = [vp, i32, vp, vp, i32, ctypes.c_float, vp, sz, vp]
        L.ctis_batch_solve_iterate.restype = st
        L.ctis_em_vjp.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, sz, vp]
        L.ctis_em_vjp.restype = st
        L.ctis_plan_set_values.argtypes = [vp, vp, vp]
        L.ctis_plan_set_values.restype = st
        L.ctis_batch_em_vjp.argtypes = [vp, vp, vp, vp, vp, vp, i32, vp, sz, vp]
        L.ctis_batch_em_vjp.restype = st
        L.ctis_batch_set_values.argtypes = [vp, i32, vp, vp]
        L.ctis_batch_set_values.restype = st
        L.ctis_batch_plan_entries.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.ctis_batch_plan_entries.restype = st
        L.ctis_fourier_create.argtypes = [ctypes.POINTER(vp), vp]
        L.ctis_fourier_create.restype = st
        L.ctis_fourier_destroy.argtypes = [vp]
        L.ctis_fourier_destroy.restype = None
        L.ctis_fourier_get_info.argtypes = [vp, ctypes.POINTER(_FourierInfo)]
        L.ctis_fourier_get_info.restype = st
        for fn in (L.ctis_fourier_forward, L.ctis_fourier_adjoint):
            fn.argtypes = [vp, vp, vp, vp, sz, vp]
            fn.restype = st
        L.ctis_fourier_em_iterate.argtypes = [vp, vp, vp, i32, vp, sz, vp]
        L.ctis_fourier_em_iterate.restype = st
        L.ctis_status_str.argtypes = [st]
        L.ctis_status_str.restype = ctypes.c_char_p
        L.ctis_last_error.argtypes = []
        L.ctis_last_error.restype = ctypes.c_char_p
        L.ctis_version.argtypes = []
        L.ctis_version.restype = ctypes.c_char_p
        if path is None:
            _lib = L
        return L


def _check(L, status: int, where: str):
    if status != 0:
        raise CtisError(status, where, L.ctis_last_error().decode(errors="replace"))


def _ptr(arr: np.ndarray):
    return ctypes.c_void_p(arr.ctypes.data) if arr.size else None


def _torch():
    import torch
    return torch


def _stream(torch, device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def need_tensor(x, numel: int, name: str, device):
    """Check a tensor the library will read or write through its pointer: a
    torch tensor, float32, contiguous, on ``device``, with ``numel`` elements.
    The C side cannot check sizes, so every tensor argument passes here before
    any launch; raises ValueError otherwise."""
    torch = _torch()
    if not isinstance(x, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor, got {type(x).__name__}")
    if x.dtype != torch.float32:
        raise ValueError(f"{name} must be float32, got {x.dtype}")
    if x.device != torch.device(device):
        raise ValueError(f"{name} must be on {device}, got {x.device}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if x.numel() != int(numel):
        raise ValueError(f"{name} must have {int(numel)} elements, got {x.numel()}")
    return x


def need_workspace(ws, nbytes: int, name: str, device):
    """A workspace tensor: contiguous, on ``device``, at least ``nbytes`` bytes."""
    torch = _torch()
    if not isinstance(ws, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor, got {type(ws).__name__}")
    if ws.device != torch.device(device):
        raise ValueError(f"{name} must be on {device}, got {ws.device}")
    if not ws.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    have = ws.numel() * ws.element_size()
    if have < int(nbytes):
        raise ValueError(f"{name} needs {int(nbytes)} bytes, got {have}")
    return ctypes.c_void_p(ws.data_ptr()), have


class Plan:
    """One geometry and one set of calibration images, on the current GPU.

    ``lambda_ptr``/``fpa_index``/``value`` describe the calibration image of
    field-stop pixel (0, 0) for every wavelength as COO (see include/ctis.h).
    """

    def __init__(self, a, alpha, w, gamma, xi, lambda_ptr, fpa_index, value, *,
                 box: int = 0, host_only: bool = False, keep_zeros: bool = False, tile_path: bool = False,
                 region: int = 0, device=None):
        self._L = load_library()
        self._handle = None
        ptr = np.ascontiguousarray(lambda_ptr, dtype=np.int64)
        idx = np.ascontiguousarray(fpa_index, dtype=np.int32)
        val = np.ascontiguousarray(value, dtype=np.float32)
        if ptr.ndim != 1 or ptr.size != int(w) + 1:
            raise ValueError("lambda_ptr must have w+1 entries")
        if ptr.size and ptr[-1] > min(idx.size, val.size):
            raise ValueError("fpa_index/value shorter than lambda_ptr[w]")
        if region and tuple(region) not in REGION_SHAPES[1:]:
            raise ValueError(f"region must be one of {REGION_SHAPES[1:]} (pixels along gamma, xi) or 0")
        flags = (CTIS_PLAN_BOX(box) | (CTIS_PLAN_HOST_ONLY if host_only else 0)
                 | (CTIS_PLAN_KEEP_ZEROS if keep_zeros else 0) | (CTIS_PLAN_TILE_PATH if tile_path else 0)
                 | (REGION_SHAPES.index(tuple(region)) << 12 if region else 0))
        self.device = None
        if not host_only:
            torch = _torch()
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible: a device plan needs an MI355X (use host_only=True to inspect)")
            self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                       else torch.device(device).index or 0)
            torch.cuda.set_device(self.device)
        h = ctypes.c_void_p()
        st = self._L.ctis_plan_create(ctypes.byref(h), int(a), int(alpha), int(w), int(gamma), int(xi),
                                      _ptr(ptr), _ptr(idx), _ptr(val), flags)
        _check(self._L, st, "ctis_plan_create")
        self._handle = h
        self._info_cache = self._info()
        self._info_stale = False
        # sizes and layout never change after creation; `info` re-reads the
        # sign flag after set_values (which synchronises the device)
        self.sizes = self._info_cache
        self.shape_f = (self.sizes.w, self.sizes.alpha, self.sizes.a)
        self.shape_g = (self.sizes.xi, self.sizes.gamma)

    @classmethod
    def from_case(cls, case, **kw):
        g = case.geometry
        return cls(g.a, g.alpha, g.w, g.gamma, g.xi, case.lambda_ptr, case.fpa_index, case.value, **kw)

    # -- lifetime -----------------------------------------------------------------
    def close(self):
        if self._handle:
            if self.device is not None:
                _torch().cuda.synchronize(self.device)
            self._L.ctis_plan_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- inspection -----------------------------------------------------------------
    @property
    def info(self) -> PlanInfo:
        """Sizes and layout decisions (re-read after set_values, which can
        change the sign flag)."""
        if self._info_stale:
            self._info_cache = self._info()
            self._info_stale = False
        return self._info_cache

    def _info(self) -> PlanInfo:
        inf = _Info()
        _check(self._L, self._L.ctis_plan_get_info(self._handle, ctypes.byref(inf)), "ctis_plan_get_info")
        d = {k: getattr(inf, k) for k, _ in _Info._fields_}
        d["nonnegative"] = bool(d["nonnegative"])
        d["dropped"] = bool(d["dropped"])
        d["em_region_path"] = bool(d["em_region_path"])
        return PlanInfo(**d)

    def lambda_sums(self) -> np.ndarray:
        out = np.empty(self.sizes.w, np.float32)
        _check(self._L, self._L.ctis_plan_lambda_sums(self._handle, _ptr(out)), "ctis_plan_lambda_sums")
        return out

    def boxes(self):
        """(box_lambda[nb], box_rc[nb, 2], box_values[nb, B, B] indexed [k, dc, dr])."""
        nb, B = self.sizes.n_boxes, self.sizes.box
        lam = np.empty(nb, np.int32)
        rc = np.empty(2 * nb, np.int32)
        vals = np.empty(nb * B * B, np.float32)
        _check(self._L, self._L.ctis_plan_export_boxes(self._handle, _ptr(lam), _ptr(rc), _ptr(vals)),
               "ctis_plan_export_boxes")
        return lam, rc.reshape(nb, 2), vals.reshape(nb, B, B)

    def worklist(self):
        """(tile_ptr[n_tiles+1], item_box[n_items])."""
        tp = np.empty(self.sizes.n_tiles + 1, np.int32)
        ib = np.empty(self.sizes.n_items, np.int32)
        _check(self._L, self._L.ctis_plan_export_worklist(self._handle, _ptr(tp), _ptr(ib)),
               "ctis_plan_export_worklist")
        return tp, ib

    def regions(self):
        """(region_ptr[n_regions+1], item_box[n_region_items]) of the region path."""
        rp = np.empty(self.sizes.n_regions + 1, np.int32)
        ib = np.empty(self.sizes.n_region_items, np.int32)
        _check(self._L, self._L.ctis_plan_export_regions(self._handle, _ptr(rp), _ptr(ib)),
               "ctis_plan_export_regions")
        return rp, ib

    # -- compute ----------------------------------------------------------------------
    def _need_device(self):
        if self.device is None:
            raise RuntimeError("host-only plan: no compute")
        if not self._handle:
            raise RuntimeError("plan is closed")

    def _dev_tensor(self, x, numel, name):
        torch = _torch()
        if not isinstance(x, torch.Tensor):
            x = torch.as_tensor(np.asarray(x, dtype=np.float32))
        x = x.to(device=self.device, dtype=torch.float32)
        if x.numel() != numel:
            raise ValueError(f"{name} must have {numel} elements, got {x.numel()}")
        return x.contiguous()

    def forward(self, f, out=None):
        """g = H f.  f: (w, alpha, a) float32 on the plan's GPU -> (xi, gamma)."""
        self._need_device()
        torch = _torch()
        f = self._dev_tensor(f, self.sizes.m, "f")
        if out is None:
            out = torch.empty(self.shape_g, dtype=torch.float32, device=self.device)
        need_tensor(out, self.sizes.n, "out", self.device)
        st = self._L.ctis_forward(self._handle, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  _stream(torch, self.device))
        _check(self._L, st, "ctis_forward")
        return out

    def adjoint(self, r, out=None):
        """z = H^T r.  r: (xi, gamma) float32 on the plan's GPU -> (w, alpha, a)."""
        self._need_device()
        torch = _torch()
        r = self._dev_tensor(r, self.sizes.n, "r")
        if out is None:
            out = torch.empty(self.shape_f, dtype=torch.float32, device=self.device)
        need_tensor(out, self.sizes.m, "out", self.device)
        st = self._L.ctis_adjoint(self._handle, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  _stream(torch, self.device))
        _check(self._L, st, "ctis_adjoint")
        return out

    def workspace(self):
        torch = _torch()
        nbytes = self.sizes.workspace_bytes
        return torch.empty(max(nbytes // 4, 64), dtype=torch.float32, device=self.device)

    def _ws(self, workspace, nbytes=None):
        return need_workspace(workspace, self.sizes.workspace_bytes if nbytes is None else nbytes, "workspace",
                              self.device)

    def em_forward_ratio(self, f, g, workspace):
        """u = g / (H f) into the first n floats of the workspace (one EM half)."""
        self._need_device()
        torch = _torch()
        need_tensor(f, self.sizes.m, "f", self.device)
        need_tensor(g, self.sizes.n, "g", self.device)
        wp, wb = self._ws(workspace)
        st = self._L.ctis_em_forward_ratio(self._handle, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                           wp, wb, _stream(torch, self.device))
        _check(self._L, st, "ctis_em_forward_ratio")
        return workspace[: self.sizes.n].view(self.shape_g)

    def em_adjoint_update(self, workspace, f_in, f_out):
        """f_out = f_in * (H^T u) / h with u from the workspace (the other EM half)."""
        self._need_device()
        torch = _torch()
        need_tensor(f_in, self.sizes.m, "f_in", self.device)
        need_tensor(f_out, self.sizes.m, "f_out", self.device)
        wp, wb = self._ws(workspace)
        st = self._L.ctis_em_adjoint_update(self._handle, wp, wb, ctypes.c_void_p(f_in.data_ptr()),
                                            ctypes.c_void_p(f_out.data_ptr()), _stream(torch, self.device))
        _check(self._L, st, "ctis_em_adjoint_update")
        return f_out

    def em(self, g, iters: int, f0=None, f=None, workspace=None, start: str = "ones"):
        """EM iterations.  Returns f after ``iters`` updates of f0.  Without f0
        the start is all ones (``start="ones"``) or H^T g (``start="adjoint"``;
        Sec. 2 names both).  If ``f`` is given it is updated in place (and
        returned) and ``f0``/``start`` are ignored."""
        self._need_device()
        torch = _torch()
        g = self._dev_tensor(g, self.sizes.n, "g")
        if start not in ("ones", "adjoint"):
            raise ValueError("start must be 'ones' or 'adjoint'")
        if f is None:
            if f0 is not None:
                f = self._dev_tensor(f0, self.sizes.m, "f0").clone()
            elif start == "adjoint":
                f = self.adjoint(g)
            else:
                f = torch.ones(self.shape_f, dtype=torch.float32, device=self.device)
        else:
            need_tensor(f, self.sizes.m, "f", self.device)
        if workspace is None:
            workspace = self.workspace()
        wp, wb = self._ws(workspace)
        st = self._L.ctis_em_iterate(self._handle, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                     int(iters), wp, wb, _stream(torch, self.device))
        _check(self._L, st, "ctis_em_iterate")
        return f

    def solve_workspace(self):
        """A workspace large enough for every solver (SART's included)."""
        torch = _torch()
        return torch.empty(max(self.sizes.solve_workspace_bytes // 4, 64), dtype=torch.float32, device=self.device)

    def solve(self, g, iters: int, solver: str = "smart", relax: float = 1.0, f0=None, f=None, workspace=None):
        """``iters`` iterations of "em", "smart" (simultaneous MART) or "sart"
        (simultaneous ART kept nonnegative, relaxation ``relax`` in (0, 2)) from
        f0 (default all ones); ``f`` is updated in place if given."""
        self._need_device()
        torch = _torch()
        if solver not in SOLVERS:
            raise ValueError(f"solver must be one of {sorted(SOLVERS)}")
        g = self._dev_tensor(g, self.sizes.n, "g")
        if f is None:
            f = (torch.ones(self.shape_f, dtype=torch.float32, device=self.device) if f0 is None
                 else self._dev_tensor(f0, self.sizes.m, "f0").clone())
        else:
            need_tensor(f, self.sizes.m, "f", self.device)
        if workspace is None:
            workspace = self.solve_workspace()
        need = self.sizes.solve_workspace_bytes if solver == "sart" else self.sizes.workspace_bytes
        wp, wb = self._ws(workspace, need)
        st = self._L.ctis_solve_iterate(self._handle, SOLVERS[solver], ctypes.c_void_p(g.data_ptr()),
                                        ctypes.c_void_p(f.data_ptr()), int(iters), float(relax), wp, wb,
                                        _stream(torch, self.device))
        _check(self._L, st, "ctis_solve_iterate")
        return f

    def diagnostics(self, g, f, workspace=None, out=None):
        """(flux sum_j h_j f_j, sum g, Poisson log-likelihood, pixels with g > 0
        and H f <= 0) of the iterate f, in double precision on the GPU; `out`
        (device float64[4]) receives them without a host copy if given."""
        self._need_device()
        torch = _torch()
        g = self._dev_tensor(g, self.sizes.n, "g")
        f = self._dev_tensor(f, self.sizes.m, "f")
        ret = out is None
        if out is None:
            out = torch.empty(4, dtype=torch.float64, device=self.device)
        elif not (isinstance(out, torch.Tensor) and out.dtype == torch.float64 and out.numel() == 4
                  and out.is_contiguous() and out.device == torch.device(self.device)):
            raise ValueError("out must be a contiguous float64 tensor of 4 elements on the plan's device")
        if workspace is None:
            workspace = self.workspace()
        wp, wb = self._ws(workspace)
        st = self._L.ctis_em_diagnostics(self._handle, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), wp, wb, _stream(torch, self.device))
        _check(self._L, st, "ctis_em_diagnostics")
        if ret:
            v = out.cpu().tolist()
            return v[0], v[1], v[2], int(v[3])
        return out

    def em_static(self, g, iters: int, f):
        """EM iterations in place on ``f`` through ctis_em_iterate_static: the
        library's static device scratch stands in for the workspace (no
        allocation; calls on one device must not overlap)."""
        self._need_device()
        torch = _torch()
        g = self._dev_tensor(g, self.sizes.n, "g")
        need_tensor(f, self.sizes.m, "f", self.device)
        st = self._L.ctis_em_iterate_static(self._handle, ctypes.c_void_p(g.data_ptr()),
                                            ctypes.c_void_p(f.data_ptr()), int(iters), _stream(torch, self.device))
        _check(self._L, st, "ctis_em_iterate_static")
        return f

    # -- derivatives ------------------------------------------------------------------
    def vjp_workspace(self):
        """Workspace for em_vjp (also valid for em)."""
        torch = _torch()
        return torch.empty(max(self.sizes.vjp_workspace_bytes // 4, 64), dtype=torch.float32, device=self.device)

    def set_values(self, values):
        """New calibration values (one per entry given at creation, device
        float32) on the same structure."""
        self._need_device()
        torch = _torch()
        v = self._dev_tensor(values, self.sizes.n_entries, "values") if self.sizes.n_entries else None
        st = self._L.ctis_plan_set_values(self._handle, ctypes.c_void_p(v.data_ptr()) if v is not None else None,
                                          _stream(torch, self.device))
        _check(self._L, st, "ctis_plan_set_values")
        self._info_stale = True

    def em_vjp(self, g, f, y, df=None, dvalues=None, accumulate: bool = False, workspace=None):
        """Reverse-mode derivative of one EM iteration at input f for the
        upstream gradient y = dL/df'.  Returns dL/df (into ``df`` if given; it
        may be ``y`` itself) and, if ``dvalues`` is given, writes (or adds, with
        ``accumulate``) dL/dv per calibration entry into it."""
        self._need_device()
        torch = _torch()
        g = self._dev_tensor(g, self.sizes.n, "g")
        f = self._dev_tensor(f, self.sizes.m, "f")
        y = self._dev_tensor(y, self.sizes.m, "y")
        if df is None:
            df = torch.empty(self.shape_f, dtype=torch.float32, device=self.device)
        need_tensor(df, self.sizes.m, "df", self.device)
        if workspace is None:
            workspace = self.vjp_workspace()
        wp, wb = self._ws(workspace, self.sizes.vjp_workspace_bytes)
        dvp = None
        if dvalues is not None:
            need_tensor(dvalues, self.sizes.n_entries, "dvalues", self.device)
            dvp = ctypes.c_void_p(dvalues.data_ptr())
        st = self._L.ctis_em_vjp(self._handle, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                 ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(df.data_ptr()), dvp,
                                 1 if accumulate else 0, wp, wb, _stream(torch, self.device))
        _check(self._L, st, "ctis_em_vjp")
        return df


class Batch:
    """Frames with their own plans (uneven sizes), reconstructed together: one
    forward+ratio and one adjoint+update launch per EM iteration for all
    frames.  Frame k's datacube is f_all[f_offsets[k] : f_offsets[k] + m_k]
    and its image g_all[g_offsets[k] : ...] (see include/ctis.h).

    Launch options (all results agree with the oracle; only speed differs):
    waves_forward / waves_adjoint: waves per workgroup of the tile kernels
    (1 = a wavefront per unit walking all its boxes, 0 = built-in);
    waves_region: waves per workgroup of the region forward; persistent:
    workgroups walk the unit list; tile_path: EM forward on FPA tiles even
    where the region path applies; region_solo: region forward with a lane
    group per region (4, 8 or 16 regions per wavefront by region size)."""

    def __init__(self, plans, waves_forward: int = 0, waves_adjoint: int = 0, persistent: bool = False,
                 waves_region: int = 0, tile_path: bool = False, region_solo: bool = False):
        self._L = load_library()
        self._handle = None
        self.plans = list(plans)
        if not self.plans:
            raise ValueError("a batch needs at least one plan")
        for p in self.plans:
            p._need_device()
        self.device = self.plans[0].device
        arr = (ctypes.c_void_p * len(self.plans))(*[p._handle.value for p in self.plans])
        for name, v, hi in (("waves_forward", waves_forward, 31), ("waves_adjoint", waves_adjoint, 31),
                            ("waves_region", waves_region, 15)):
            if not 0 <= int(v) <= hi:
                raise ValueError(f"{name} must be in 0..{hi}")
        flags = (int(waves_forward) | (int(waves_adjoint) << 5) | (int(waves_region) << 11)
                 | (CTIS_BATCH_PERSISTENT if persistent else 0) | (CTIS_BATCH_TILE_PATH if tile_path else 0)
                 | (CTIS_BATCH_REGION_SOLO if region_solo else 0))
        h = ctypes.c_void_p()
        _check(self._L, self._L.ctis_batch_create(ctypes.byref(h), ctypes.cast(arr, ctypes.c_void_p),
                                                  len(self.plans), flags), "ctis_batch_create")
        self._handle = h
        inf = _BatchInfo()
        _check(self._L, self._L.ctis_batch_get_info(self._handle, ctypes.byref(inf)), "ctis_batch_get_info")
        self.info = {k: getattr(inf, k) for k, _ in _BatchInfo._fields_}
        m = np.array([p.sizes.m for p in self.plans], np.int64)
        n = np.array([p.sizes.n for p in self.plans], np.int64)
        self.f_offsets = np.concatenate([[0], np.cumsum(m)])
        self.g_offsets = np.concatenate([[0], np.cumsum(n)])

    def close(self):
        if self._handle:
            _torch().cuda.synchronize(self.device)
            self._L.ctis_batch_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def frame_f(self, f_all, k):
        return f_all[self.f_offsets[k]:self.f_offsets[k + 1]].view(self.plans[k].shape_f)

    def frame_g(self, g_all, k):
        return g_all[self.g_offsets[k]:self.g_offsets[k + 1]].view(self.plans[k].shape_g)

    def pack_g(self, images):
        torch = _torch()
        return torch.cat([torch.as_tensor(x, dtype=torch.float32, device=self.device).reshape(-1) for x in images])

    def workspace(self):
        torch = _torch()
        return torch.empty(max(self.info["workspace_bytes"] // 4, 64), dtype=torch.float32, device=self.device)

    @property
    def m_total(self) -> int:
        return int(self.f_offsets[-1])

    @property
    def n_total(self) -> int:
        return int(self.g_offsets[-1])

    def _ws(self, workspace, nbytes):
        return need_workspace(workspace, nbytes, "workspace", self.device)

    def forward(self, f_all, out=None):
        torch = _torch()
        need_tensor(f_all, self.m_total, "f_all", self.device)
        if out is None:
            out = torch.empty(self.n_total, dtype=torch.float32, device=self.device)
        need_tensor(out, self.n_total, "out", self.device)
        st = self._L.ctis_batch_forward(self._handle, ctypes.c_void_p(f_all.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        _stream(torch, self.device))
        _check(self._L, st, "ctis_batch_forward")
        return out

    def adjoint(self, r_all, out=None):
        torch = _torch()
        need_tensor(r_all, self.n_total, "r_all", self.device)
        if out is None:
            out = torch.empty(self.m_total, dtype=torch.float32, device=self.device)
        need_tensor(out, self.m_total, "out", self.device)
        st = self._L.ctis_batch_adjoint(self._handle, ctypes.c_void_p(r_all.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        _stream(torch, self.device))
        _check(self._L, st, "ctis_batch_adjoint")
        return out

    def em(self, g_all, iters: int, f_all=None, workspace=None, start: str = "ones"):
        """EM of every frame in place on f_all (default: a new f_all, all ones
        or, with ``start="adjoint"``, H^T g of each frame)."""
        torch = _torch()
        if start not in ("ones", "adjoint"):
            raise ValueError("start must be 'ones' or 'adjoint'")
        need_tensor(g_all, self.n_total, "g_all", self.device)
        if f_all is None:
            if start == "adjoint":
                f_all = self.adjoint(g_all)
            else:
                f_all = torch.ones(self.m_total, dtype=torch.float32, device=self.device)
        need_tensor(f_all, self.m_total, "f_all", self.device)
        if workspace is None:
            workspace = self.workspace()
        wp, wb = self._ws(workspace, self.info["workspace_bytes"])
        st = self._L.ctis_batch_em_iterate(self._handle, ctypes.c_void_p(g_all.data_ptr()),
                                           ctypes.c_void_p(f_all.data_ptr()), int(iters), wp, wb,
                                           _stream(torch, self.device))
        _check(self._L, st, "ctis_batch_em_iterate")
        return f_all

    def solve_workspace(self):
        """A workspace large enough for every solver (SART's included)."""
        torch = _torch()
        return torch.empty(max(self.info["solve_workspace_bytes"] // 4, 64), dtype=torch.float32,
                           device=self.device)

    def solve(self, g_all, iters: int, solver: str = "smart", relax: float = 1.0, f_all=None, workspace=None):
        """Plan.solve for every frame at once (f_all updated in place if given,
        else a new all-ones start)."""
        torch = _torch()
        if solver not in SOLVERS:
            raise ValueError(f"solver must be one of {sorted(SOLVERS)}")
        need_tensor(g_all, self.n_total, "g_all", self.device)
        if f_all is None:
            f_all = torch.ones(self.m_total, dtype=torch.float32, device=self.device)
        need_tensor(f_all, self.m_total, "f_all", self.device)
        if workspace is None:
            workspace = self.solve_workspace()
        need = self.info["solve_workspace_bytes"] if solver == "sart" else self.info["workspace_bytes"]
        wp, wb = self._ws(workspace, need)
        st = self._L.ctis_batch_solve_iterate(self._handle, SOLVERS[solver], ctypes.c_void_p(g_all.data_ptr()),
                                              ctypes.c_void_p(f_all.data_ptr()), int(iters), float(relax), wp, wb,
                                              _stream(torch, self.device))
        _check(self._L, st, "ctis_batch_solve_iterate")
        return f_all

    def em_forward_ratio(self, f_all, g_all, workspace):
        """u = g / (H f) of every frame into the start of the workspace (one EM
        half of all frames)."""
        torch = _torch()
        need_tensor(f_all, self.m_total, "f_all", self.device)
        need_tensor(g_all, self.n_total, "g_all", self.device)
        wp, wb = self._ws(workspace, self.info["workspace_bytes"])
        st = self._L.ctis_batch_em_forward_ratio(self._handle, ctypes.c_void_p(f_all.data_ptr()),
                                                 ctypes.c_void_p(g_all.data_ptr()), wp, wb, _stream(torch, self.device))
        _check(self._L, st, "ctis_batch_em_forward_ratio")
        return workspace[: self.n_total]

    def em_adjoint_update(self, workspace, f_in, f_out):
        """f_out = f_in * (H^T u) / h of every frame, u from the workspace (the
        other EM half)."""
        torch = _torch()
        need_tensor(f_in, self.m_total, "f_in", self.device)
        need_tensor(f_out, self.m_total, "f_out", self.device)
        wp, wb = self._ws(workspace, self.info["workspace_bytes"])
        st = self._L.ctis_batch_em_adjoint_update(self._handle, wp, wb, ctypes.c_void_p(f_in.data_ptr()),
                                                  ctypes.c_void_p(f_out.data_ptr()), _stream(torch, self.device))
        _check(self._L, st, "ctis_batch_em_adjoint_update")
        return f_out

    # -- derivatives ------------------------------------------------------------------
    def vjp_workspace(self):
        torch = _torch()
        return torch.empty(max(self.info["vjp_workspace_bytes"] // 4, 64), dtype=torch.float32, device=self.device)

    def plan_entries(self, k: int):
        """(offset, count) of frame k's plan's entries in the batch's value arrays."""
        off, cnt = ctypes.c_int64(), ctypes.c_int64()
        _check(self._L, self._L.ctis_batch_plan_entries(self._handle, int(k), ctypes.byref(off), ctypes.byref(cnt)),
               "ctis_batch_plan_entries")
        return off.value, cnt.value

    def set_values(self, k: int, values):
        """New values for the plan of frame k (and the frames sharing it)."""
        torch = _torch()
        v = torch.as_tensor(values, dtype=torch.float32, device=self.device).contiguous()
        need_tensor(v, self.plan_entries(k)[1], "values", self.device)
        st = self._L.ctis_batch_set_values(self._handle, int(k), ctypes.c_void_p(v.data_ptr()) if v.numel() else None,
                                           _stream(torch, self.device))
        _check(self._L, st, "ctis_batch_set_values")

    def em_vjp(self, g_all, f_all, y_all, df_all=None, dvalues=None, accumulate: bool = False, workspace=None):
        """Batch form of Plan.em_vjp; dvalues holds the entries of the batch's
        distinct plans back to back (see plan_entries)."""
        torch = _torch()
        need_tensor(g_all, self.n_total, "g_all", self.device)
        need_tensor(f_all, self.m_total, "f_all", self.device)
        need_tensor(y_all, self.m_total, "y_all", self.device)
        if df_all is None:
            df_all = torch.empty(self.m_total, dtype=torch.float32, device=self.device)
        need_tensor(df_all, self.m_total, "df_all", self.device)
        if workspace is None:
            workspace = self.vjp_workspace()
        wp, wb = self._ws(workspace, self.info["vjp_workspace_bytes"])
        dvp = None
        if dvalues is not None:
            need_tensor(dvalues, self.info["n_entries"], "dvalues", self.device)
            dvp = ctypes.c_void_p(dvalues.data_ptr())
        st = self._L.ctis_batch_em_vjp(self._handle, ctypes.c_void_p(g_all.data_ptr()),
                                       ctypes.c_void_p(f_all.data_ptr()), ctypes.c_void_p(y_all.data_ptr()),
                                       ctypes.c_void_p(df_all.data_ptr()), dvp, 1 if accumulate else 0,
                                       wp, wb, _stream(torch, self.device))
        _check(self._L, st, "ctis_batch_em_vjp")
        return df_all


class Fourier:
    """The Fourier (WBH) projections of a plan: spectra of its calibration
    and FFT-based forward, adjoint and EM (see include/ctis.h).  The plan must
    outlive this object."""

    def __init__(self, plan: Plan):
        self._L = load_library()
        self._handle = None
        plan._need_device()
        self.plan = plan
        self.device = plan.device
        h = ctypes.c_void_p()
        _check(self._L, self._L.ctis_fourier_create(ctypes.byref(h), plan._handle), "ctis_fourier_create")
        self._handle = h
        inf = _FourierInfo()
        _check(self._L, self._L.ctis_fourier_get_info(self._handle, ctypes.byref(inf)), "ctis_fourier_get_info")
        self.info = {k: getattr(inf, k) for k, _ in _FourierInfo._fields_}

    def close(self):
        if self._handle:
            _torch().cuda.synchronize(self.device)
            self._L.ctis_fourier_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self):
        torch = _torch()
        return torch.empty(max(self.info["workspace_bytes"] // 4, 64), dtype=torch.float32, device=self.device)

    def forward(self, f, out=None, workspace=None):
        torch = _torch()
        f = self.plan._dev_tensor(f, self.plan.sizes.m, "f")
        if out is None:
            out = torch.empty(self.plan.shape_g, dtype=torch.float32, device=self.device)
        need_tensor(out, self.plan.sizes.n, "out", self.device)
        ws = self.workspace() if workspace is None else workspace
        wp, wb = need_workspace(ws, self.info["workspace_bytes"], "workspace", self.device)
        st = self._L.ctis_fourier_forward(self._handle, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          wp, wb, _stream(torch, self.device))
        _check(self._L, st, "ctis_fourier_forward")
        return out

    def adjoint(self, r, out=None, workspace=None):
        torch = _torch()
        r = self.plan._dev_tensor(r, self.plan.sizes.n, "r")
        if out is None:
            out = torch.empty(self.plan.shape_f, dtype=torch.float32, device=self.device)
        need_tensor(out, self.plan.sizes.m, "out", self.device)
        ws = self.workspace() if workspace is None else workspace
        wp, wb = need_workspace(ws, self.info["workspace_bytes"], "workspace", self.device)
        st = self._L.ctis_fourier_adjoint(self._handle, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          wp, wb, _stream(torch, self.device))
        _check(self._L, st, "ctis_fourier_adjoint")
        return out

    def em(self, g, iters: int, f0=None, f=None, workspace=None):
        torch = _torch()
        g = self.plan._dev_tensor(g, self.plan.sizes.n, "g")
        if f is None:
            f = (torch.ones(self.plan.shape_f, dtype=torch.float32, device=self.device) if f0 is None
                 else self.plan._dev_tensor(f0, self.plan.sizes.m, "f0").clone())
        need_tensor(f, self.plan.sizes.m, "f", self.device)
        ws = self.workspace() if workspace is None else workspace
        wp, wb = need_workspace(ws, self.info["workspace_bytes"], "workspace", self.device)
        st = self._L.ctis_fourier_em_iterate(self._handle, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                             int(iters), wp, wb, _stream(torch, self.device))
        _check(self._L, st, "ctis_fourier_em_iterate")
        return f
