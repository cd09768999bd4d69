"""Autotuner for batched reconstructions of frames of uneven shapes.

Candidate configurations of a batch:

* forward projection: the region path with each region shape of a group of
  16 lanes (16 x 16, 32 x 8 and 8 x 32 FPA pixels, i.e. two fast-axis widths
  and two slow-axis heights around the square one) and 2, 3 or 4 wavefronts
  per workgroup sharing each region's boxes; or with a lane group per
  region ("solo"), in those shapes (four regions per wavefront) and in the
  smaller ones of groups of 8 and 4 lanes (16 x 8, 8 x 16: eight regions
  per wavefront; 8 x 8: sixteen), which follow the edges of small box
  images more closely; or the tile path (64 x 16 FPA tiles) with 1 (a
  wavefront per tile), 4, 8 or 16.  (The cooperative kernel is not tried
  with the smaller regions: with 8 or 16 groups per wavefront the short box
  lists of a batch leave most of a pass's groups on empty records.)
* one workgroup per work unit, or a persistent grid whose workgroups walk
  the unit list;
* then, with the winning forward setup, the back projection's waves per
  workgroup: the built-in choice, 4 or 8 waves sharing a unit's boxes, or a
  wavefront per unit (1);
* then the calibration box side B (the window halo is B - 1 pixels) one
  below and one above the plan's own choice, with the winning launch setup.

Arrangements are tuned and timed whole: every frame in one batch with one
configuration (one launch per kernel and EM iteration); a configuration per
frame shape (field stop, wavelengths, FPA), each tuned on its shape's
frames, with one batch per distinct winner run back to back; and the same
two run as concurrent groups -- the uniform configuration over two batches
of about equal work, or the per-shape batches -- each group on a stream of
its own (default priority) with its own slice of the workspace, so that one
group's forward projection runs beside another's back projection and each
fills the other's waits on memory (frames are independent: no exchange).
The fastest arrangement is kept (`TunedBatch`).  Timing uses HIP events on
the current stream.  Nothing here changes results beyond the summation order
of the projections.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import ctis

REGION_SHAPES = ((16, 16), (32, 8), (8, 32))
SOLO_SHAPES = REGION_SHAPES + ((16, 8), (8, 16), (8, 8))
REGION_WAVES = (2, 3, 4)
TILE_WAVES = (1, 4, 8, 16)
ADJOINT_WAVES = (1, 4, 8)


@dataclasses.dataclass(frozen=True)
class Choice:
    """A launch configuration of one batch."""
    path: str                     # "region", "solo" (region, a lane group per region) or "tile"
    shape: tuple | None           # region shape (pixels along gamma, xi); None on the tile path
    waves: int                    # wavefronts per forward workgroup (1: a wave per unit)
    persistent: bool
    box: int                      # calibration box side B (0: the plan's choice)
    adj_waves: int = 0            # back projection's waves per workgroup (0: built-in, 1: a wave per unit)

    def label(self) -> str:
        sh = f"{self.shape[0]}x{self.shape[1]}" if self.shape else "64x16"
        return (f"{self.path} {sh} W{self.waves}{' persistent' if self.persistent else ''}"
                f" adjoint W{self.adj_waves if self.adj_waves else 'auto'} B{self.box if self.box else 'auto'}")

    @classmethod
    def parse(cls, label: str) -> "Choice":
        """The Choice a label() string names, e.g. "tile 64x16 W4 adjoint W1 Bauto"."""
        t = label.split()
        try:
            path, sh, w = t[0], t[1], t[2]
            persistent = "persistent" in t
            rest = t[3 + persistent:]
            if path not in ("region", "solo", "tile") or rest[0] != "adjoint" or not w.startswith("W"):
                raise ValueError
            shape = None if path == "tile" else tuple(int(x) for x in sh.split("x"))
            aw = 0 if rest[1] == "Wauto" else int(rest[1][1:])
            box = 0 if rest[2] == "Bauto" else int(rest[2][1:])
            return cls(path, shape, int(w[1:]), persistent, box, aw)
        except (IndexError, ValueError):
            raise ValueError(f"not a launch choice: {label!r}") from None


def _time_em(torch, batch, g_all, iters: int, reps: int, graph: bool = False) -> float:
    """Best time (ms) of one EM iteration of the batch over `reps` runs of
    `iters` iterations, launched from the stream or (``graph``) replayed from
    a HIP graph of the run, as a solve is launched in production (concurrent
    arrangements only pay off there: launched one by one, the host's launch
    rate bounds them)."""
    ws = batch.workspace()
    f = torch.ones(batch.m_total, dtype=torch.float32, device=batch.device)
    batch.em(g_all, 1, f_all=f, workspace=ws)          # warm-up (code objects, caches)
    run = lambda: batch.em(g_all, iters, f_all=f, workspace=ws)
    if graph:
        s = torch.cuda.Stream(device=batch.device)
        s.wait_stream(torch.cuda.current_stream(batch.device))
        with torch.cuda.stream(s):
            run()                                      # outside the capture first
        torch.cuda.current_stream(batch.device).wait_stream(s)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            run()
        run = gr.replay
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        f.fill_(1.0)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / iters)
    return best


def _plans(cases, choice: Choice, cache: dict):
    """Plans of the cases for a choice's box side and region shape (cached)."""
    key = (choice.box, choice.shape)
    if key not in cache:
        kw = {"box": choice.box}
        if choice.shape:
            kw["region"] = choice.shape
        cache[key] = [ctis.Plan.from_case(c, **kw) for c in cases]
    return cache[key]


def _batch(plans, choice: Choice):
    if choice.path == "solo":
        return ctis.Batch(plans, region_solo=True, waves_adjoint=choice.adj_waves, persistent=choice.persistent)
    if choice.path == "region":
        return ctis.Batch(plans, waves_region=choice.waves, waves_adjoint=choice.adj_waves,
                          persistent=choice.persistent)
    return ctis.Batch(plans, waves_forward=choice.waves, waves_adjoint=choice.adj_waves,
                      persistent=choice.persistent, tile_path=True)


def _candidates(region_ok: bool, box: int):
    out = []
    for pe in (False, True):
        if region_ok:
            out += [Choice("region", sh, w, pe, 0) for sh in REGION_SHAPES for w in REGION_WAVES]
            out += [Choice("solo", sh, 4, pe, 0) for sh in SOLO_SHAPES]
        out += [Choice("tile", None, w, pe, 0) for w in TILE_WAVES if w <= (16 if box <= 5 else 8)]
    return out


def tune_frames(torch, cases, images, iters: int, reps: int, table: list, cls: str):
    """Fastest Choice for one batch over `cases`; appends every timing to
    `table`."""
    cache = {}
    base = _plans(cases, Choice("tile", None, 4, False, 0), cache)
    B0 = base[0].info.box
    best = None

    def trial(choice):
        nonlocal best
        plans = _plans(cases, choice, cache)
        if choice.path in ("region", "solo") and not all(p.info.em_region_path for p in plans):
            return
        if len({p.info.box for p in plans}) != 1:
            return
        try:
            b = _batch(plans, choice)
        except ctis.CtisError:            # a launch setup the box side does not allow
            return
        g_all = b.pack_g(images)
        ms = _time_em(torch, b, g_all, iters, reps)
        b.close()
        table.append({"frames": cls, "choice": choice.label(), "ms_per_iter": ms})
        if best is None or ms < best[0]:
            best = (ms, choice)

    region_ok = all(p.info.em_region_path for p in base)
    for ch in _candidates(region_ok, B0):
        trial(ch)
    # the back projection's launch setup with the winning forward one
    _, chf = best
    for wa in ADJOINT_WAVES:
        if wa <= (16 if B0 <= 5 else 8):
            trial(dataclasses.replace(chf, adj_waves=wa))
    # the halo: box sides around the plan's choice with the winning launch setup
    ms0, ch0 = best
    for B in (B0 - 1, B0 + 1):
        if 1 <= B <= 8:
            trial(dataclasses.replace(ch0, box=B))
    for plans in cache.values():
        for p in plans:
            p.close()
    return best[1], best[0]


MAX_CONCURRENT = 4   # streams of concurrent groups (the hardware queues a process gets by default)


class TunedBatch:
    """Frames of uneven shapes, reconstructed as one batch per group (a tuned
    configuration and its frames), the groups one after another or, with
    ``concurrent``, side by side on streams of their own.  Buffers are packed
    in the tuned frame order: frame k (original index) holds
    f_all[f_offsets[pos[k]] : ...] with pos the inverse of `order`."""

    def __init__(self, cases, groups, concurrent: bool = False):
        # groups: list of (choice, [original frame indices])
        if concurrent and not 1 <= len(groups) <= MAX_CONCURRENT:
            raise ValueError(f"concurrent arrangements take 1 to {MAX_CONCURRENT} groups")
        self.concurrent = bool(concurrent) and len(groups) > 1
        self.groups = []
        self.order = [k for _, idx in groups for k in idx]
        self.pos = np.empty(len(self.order), np.int64)
        self.pos[self.order] = np.arange(len(self.order))
        f0 = g0 = 0
        self.f_offsets, self.g_offsets = [0], [0]
        for choice, idx in groups:
            kw = {"box": choice.box}
            if choice.shape:
                kw["region"] = choice.shape
            plans = [ctis.Plan.from_case(cases[k], **kw) for k in idx]
            b = _batch(plans, choice)
            self.groups.append((choice, idx, plans, b, f0, g0))
            for p in plans:
                f0 += p.sizes.m
                g0 += p.sizes.n
                self.f_offsets.append(f0)
                self.g_offsets.append(g0)
        self.f_offsets = np.array(self.f_offsets, np.int64)
        self.g_offsets = np.array(self.g_offsets, np.int64)
        self.device = self.groups[0][3].device
        # workspace slices: one shared by sequential groups, one per group
        # (256-byte aligned) for concurrent ones
        need = [b.info["workspace_bytes"] for _, _, _, b, _, _ in self.groups]
        if self.concurrent:
            self.ws_offsets = list(np.cumsum([0] + [(n + 255) // 256 * 256 for n in need[:-1]]))
            self.ws_bytes = int(self.ws_offsets[-1] + need[-1])
            torch = ctis._torch()
            self.streams = [torch.cuda.Stream(device=self.device) for _ in self.groups]
        else:
            self.ws_offsets = [0] * len(need)
            self.ws_bytes = max(need)
            self.streams = None

    @property
    def m_total(self) -> int:
        return int(self.f_offsets[-1])

    def pack_g(self, images):
        """Images of the frames (original order) packed in the tuned order."""
        torch = ctis._torch()
        return torch.cat([torch.as_tensor(images[k], dtype=torch.float32, device=self.device).reshape(-1)
                          for k in self.order])

    def frame_f(self, f_all, k):
        """View of original frame k's datacube in a packed f_all."""
        j = int(self.pos[k])
        return f_all[self.f_offsets[j]:self.f_offsets[j + 1]]

    def workspace(self):
        """One workspace for every group: shared when the groups run one after
        another, a slice per group when they run concurrently."""
        torch = ctis._torch()
        return torch.empty(max((self.ws_bytes + 3) // 4, 64), dtype=torch.float32, device=self.device)

    def _ws_slice(self, workspace, j):
        off = int(self.ws_offsets[j]) // 4
        return workspace[off:off + (self.groups[j][3].info["workspace_bytes"] + 3) // 4]

    def em(self, g_all, iters: int, f_all=None, workspace=None):
        torch = ctis._torch()
        if f_all is None:
            f_all = torch.ones(self.m_total, dtype=torch.float32, device=self.device)
        if workspace is None:
            workspace = self.workspace()
        if workspace.numel() * 4 < self.ws_bytes:
            raise ValueError(f"workspace of {workspace.numel() * 4} bytes; the arrangement needs {self.ws_bytes}")
        if not self.concurrent:
            for _, _, _, b, f0, g0 in self.groups:
                b.em(g_all[g0:g0 + b.n_total], iters, f_all=f_all[f0:f0 + b.m_total], workspace=workspace)
            return f_all
        # fork: every group's stream waits for the work queued so far, runs
        # its batch, and the current stream waits for all of them (HIP graph
        # capture records the branches as parallel nodes)
        cur = torch.cuda.current_stream(self.device)
        for st in self.streams:
            st.wait_stream(cur)
        for j, (st, (_, _, _, b, f0, g0)) in enumerate(zip(self.streams, self.groups)):
            with torch.cuda.stream(st):
                b.em(g_all[g0:g0 + b.n_total], iters, f_all=f_all[f0:f0 + b.m_total],
                     workspace=self._ws_slice(workspace, j))
        for st in self.streams:
            cur.wait_stream(st)
        return f_all

    def report(self):
        return [{"choice": ch.label(), "frames": len(idx)} for ch, idx, _, _, _, _ in self.groups]

    def parts(self, g_all, f_all):
        """(batch, its slice of g_all, its slice of f_all) per group."""
        return [(b, g_all[g0:g0 + b.n_total], f_all[f0:f0 + b.m_total]) for _, _, _, b, f0, g0 in self.groups]

    def close(self):
        for _, _, plans, b, _, _ in self.groups:
            b.close()
            for p in plans:
                p.close()


@dataclasses.dataclass
class TuneResult:
    batch: TunedBatch
    arrangement: str              # "uniform", "per shape", "uniform, 2 concurrent" or "per shape, concurrent"
    ms_per_iter: dict             # whole-batch EM iteration time of every arrangement (graph-launched)
    uniform: str                  # the uniform arrangement's configuration
    classes: list                 # per frame shape: its frames and the configuration tuned on them
    table: list                   # every timing


def balanced_split(cases, n: int):
    """The frames in n groups of about equal work (one EM iteration's
    multiply-adds, a alpha w times the calibration entries per wavelength):
    heaviest first, each to the lightest group so far; original order inside
    a group."""
    work = [c.geometry.a * c.geometry.alpha * int(c.lambda_ptr[-1]) for c in cases]
    load = [0] * n
    groups = [[] for _ in range(n)]
    for k in sorted(range(len(cases)), key=lambda k: (-work[k], k)):
        j = min(range(n), key=lambda j: (load[j], j))
        groups[j].append(k)
        load[j] += work[k]
    return [sorted(g) for g in groups if g]


def fixed_frames(cases, choice: Choice, split: int = 1) -> TunedBatch:
    """The frames with a given configuration (no tuning): one batch, or
    `split` concurrent batches of about equal work."""
    if split <= 1:
        return TunedBatch(cases, [(choice, list(range(len(cases))))])
    return TunedBatch(cases, [(choice, idx) for idx in balanced_split(cases, split)], concurrent=True)


def autotune_frames(cases, images, iters: int = 4, reps: int = 3) -> TuneResult:
    """Tune both arrangements and keep the faster.  `cases` carry each frame's
    geometry and calibration (workloads.Case); `images` are the frames' FPA
    images (host arrays)."""
    import torch
    table = []
    everything = list(range(len(cases)))
    uni, _ = tune_frames(torch, cases, images, iters, reps, table, "all")
    classes = {}
    for k, c in enumerate(cases):
        g = c.geometry
        classes.setdefault((g.a, g.alpha, g.w, g.gamma, g.xi), []).append(k)
    chosen = []
    for key, idx in classes.items():
        cls = "a={} alpha={} w={} FPA {}x{}".format(*key)
        choice, ms = tune_frames(torch, [cases[k] for k in idx], [images[k] for k in idx], iters, reps, table, cls)
        chosen.append(({"class": cls, "frames": len(idx), "choice": choice.label(), "ms_per_iter": ms}, choice, idx))
    merged = {}
    for _, ch, idx in chosen:
        merged.setdefault(ch, []).extend(idx)
    per_shape = [(ch, sorted(idx)) for ch, idx in merged.items()]
    arrangements = {"uniform": ([(uni, everything)], False),
                    "per shape": (per_shape, False),
                    "uniform, 2 concurrent": ([(uni, idx) for idx in balanced_split(cases, 2)], True)}
    if 1 < len(per_shape) <= MAX_CONCURRENT:
        arrangements["per shape, concurrent"] = (per_shape, True)
    timed = {}
    for name, (groups, conc) in arrangements.items():
        tb = TunedBatch(cases, groups, concurrent=conc)
        timed[name] = (_time_em(torch, tb, tb.pack_g(images), max(iters, 20), reps, graph=True), tb)
    keep = min(timed, key=lambda k: timed[k][0])
    for name, (_, tb) in timed.items():
        if name != keep:
            tb.close()
    return TuneResult(timed[keep][1], keep, {k: v[0] for k, v in timed.items()}, uni.label(),
                      [c for c, _, _ in chosen], table)
