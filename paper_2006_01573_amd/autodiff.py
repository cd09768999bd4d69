"""Differentiable unrolled EM: a ``torch.autograd.Function`` over K EM
iterations (Sec. 2 eq. (em)) whose backward runs libctis's hand-written
derivative kernels (``ctis_em_vjp`` / ``ctis_batch_em_vjp``).

Forward: set the calibration values (if given), keep the iterates
f^(1) .. f^(K) -- one checkpoint of f per iteration -- and run the K updates
with the EM kernels.  Backward: for k = K .. 1 the derivative call
recomputes that iteration's projections (H f, u, H^T u) from the checkpoint,
maps dL/df^(k+1) to dL/df^(k) in place, and adds the iteration's derivative
with respect to every calibration entry into one accumulator.  Nothing here
does arithmetic on the tensors: torch holds memory and the stream.

The operator is a ``ctis.Plan`` (one frame) or a ``ctis.Batch`` (frames back
to back; frames that share a plan share its values).  Values are one float
per calibration entry in the plan's input order (a batch: its distinct plans'
entries back to back); plans built for derivatives with respect to the values
need ``keep_zeros=True`` when a value may be zero.  The forward runs one EM
iteration per call (a checkpoint after each), so operators on the tile path
(``tile_path=True``) suit it best: the region path writes its padded copy of
f at the start of every call.
"""
from __future__ import annotations

import torch

from . import ctis


class _Op:
    """Uniform view of a Plan or a Batch."""

    def __init__(self, op):
        self.op = op
        self.is_batch = isinstance(op, ctis.Batch)
        if self.is_batch:
            self.m = int(op.f_offsets[-1])
            self.n = int(op.g_offsets[-1])
            self.n_entries = int(op.info["n_entries"])
        else:
            self.m = op.sizes.m
            self.n = op.sizes.n
            self.n_entries = op.sizes.n_entries
        self.device = op.device

    def workspace(self):
        return self.op.vjp_workspace()

    def set_values(self, values):
        if self.is_batch:
            b = self.op
            seen = set()
            for k in range(len(b.plans)):
                off, cnt = b.plan_entries(k)
                if off in seen:
                    continue
                seen.add(off)
                b.set_values(k, values[off:off + cnt])
        else:
            self.op.set_values(values)

    def em_step(self, g, f, ws):
        if self.is_batch:
            self.op.em(g, 1, f_all=f, workspace=ws)
        else:
            self.op.em(g, 1, f=f.view(self.op.shape_f), workspace=ws)

    def vjp(self, g, f, y, dv, ws):
        if self.is_batch:
            self.op.em_vjp(g, f, y, df_all=y, dvalues=dv, accumulate=True, workspace=ws)
        else:
            self.op.em_vjp(g, f, y, df=y.view(self.op.shape_f), dvalues=dv, accumulate=True, workspace=ws)


class UnrolledEM(torch.autograd.Function):
    """f^(K+1) = EM^K(f0; g, values).  Differentiable in f0 and values."""

    @staticmethod
    def forward(ctx, f0, values, g, op, iters: int):
        o = _Op(op)
        if f0.numel() != o.m or g.numel() != o.n:
            raise ValueError("f0 and g must match the operator's sizes")
        if iters < 0:
            raise ValueError("iters must be >= 0")
        g = g.detach().to(device=o.device, dtype=torch.float32).reshape(-1).contiguous()
        if values is not None:
            values = values.detach().to(device=o.device, dtype=torch.float32).reshape(-1).contiguous()
            if values.numel() != o.n_entries:
                raise ValueError(f"values must have {o.n_entries} elements")
            o.set_values(values)
        ws = o.workspace()
        f = f0.detach().to(device=o.device, dtype=torch.float32).reshape(-1).clone()
        checkpoints = []
        for _ in range(iters):
            checkpoints.append(f.clone())
            o.em_step(g, f, ws)
        ctx.o, ctx.iters, ctx.ws = o, iters, ws
        ctx.has_values = values is not None
        ctx.save_for_backward(g, values if values is not None else torch.empty(0), *checkpoints)
        return f.view(f0.shape)

    @staticmethod
    def backward(ctx, grad_out):
        o, iters, ws = ctx.o, ctx.iters, ctx.ws
        g, values, *checkpoints = ctx.saved_tensors
        if ctx.has_values:
            o.set_values(values)                 # the values this graph was recorded with
        y = grad_out.detach().to(dtype=torch.float32).reshape(-1).contiguous().clone()
        need_v = ctx.has_values and ctx.needs_input_grad[1]
        dv = torch.zeros(o.n_entries, dtype=torch.float32, device=o.device) if need_v else None
        for k in range(iters - 1, -1, -1):
            o.vjp(g, checkpoints[k], y, dv, ws)
        df0 = y.view(grad_out.shape) if ctx.needs_input_grad[0] else None
        return df0, dv, None, None, None


def unrolled_em(op, g, f0, iters: int, values=None):
    """K EM iterations on ``op`` (a ctis.Plan or ctis.Batch) from f0, with
    gradients to f0 and (if given) the calibration values."""
    return UnrolledEM.apply(f0, values, g, op, int(iters))
