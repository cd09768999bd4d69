"""Autotuner for batched reconstructions.

For a set of frames it times the batched EM iteration on the GPU for every
candidate launch configuration -- wavefronts per workgroup of the forward and
of the back-projection kernel (each wave owns one 64x16 output tile; more
waves split a tile's boxes more finely), one workgroup per work unit versus a
persistent grid -- and, if asked, for several calibration box sides B (the
window halo is B-1 pixels), and keeps the fastest.  Timing uses HIP events on
the current stream; nothing here changes results beyond the summation order
inside a tile.
"""
from __future__ import annotations

import dataclasses
import itertools

from . import ctis


@dataclasses.dataclass
class TuneResult:
    batch: "ctis.Batch"
    waves_forward: int
    waves_adjoint: int
    persistent: bool
    box: int
    ms_per_iter: float
    table: list


def _time_em(torch, batch, g_all, iters: int, reps: int) -> float:
    ws = batch.workspace()
    f = torch.ones(int(batch.f_offsets[-1]), dtype=torch.float32, device=batch.device)
    batch.em(g_all, 1, f_all=f, workspace=ws)          # warm-up (code objects, caches)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        f.fill_(1.0)
        e0.record()
        batch.em(g_all, iters, f_all=f, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / iters)
    return best


def autotune_batch(plans, g_all, iters: int = 4, reps: int = 3, waves=(4, 8, 16),
                   persistent=(False, True)) -> TuneResult:
    """Fastest launch configuration for a batch over ``plans`` (frames) with
    the packed images ``g_all``."""
    import torch
    B = plans[0].info.box
    max_w = 16 if B <= 5 else 8
    cands = [(wf, wa, pe) for wf, wa, pe in itertools.product(waves, waves, persistent)
             if wf <= max_w and wa <= max_w]
    table = []
    best = None
    for wf, wa, pe in cands:
        b = ctis.Batch(plans, waves_forward=wf, waves_adjoint=wa, persistent=pe)
        ms = _time_em(torch, b, g_all, iters, reps)
        table.append({"waves_forward": wf, "waves_adjoint": wa, "persistent": pe, "box": B, "ms_per_iter": ms})
        if best is None or ms < best[0]:
            if best is not None:
                best[1].close()
            best = (ms, b, wf, wa, pe)
        else:
            b.close()
    ms, b, wf, wa, pe = best
    return TuneResult(b, wf, wa, pe, B, ms, table)


def autotune_cases(cases, images, boxes=(0,), **kw) -> TuneResult:
    """Also tune the box side: for each B in ``boxes`` (0 = the plan's own
    choice) build the frames' plans with that B and tune the batch; return
    the fastest.  ``images`` are the frames' FPA images (host arrays)."""
    best = None
    table = []
    for B in boxes:
        plans = [ctis.Plan.from_case(c, box=B) for c in cases]
        if len({p.info.box for p in plans}) != 1:
            continue
        batch0 = ctis.Batch(plans)
        g_all = batch0.pack_g(images)
        batch0.close()
        r = autotune_batch(plans, g_all, **kw)
        table.extend(r.table)
        if best is None or r.ms_per_iter < best.ms_per_iter:
            best = r
    best.table = table
    return best
