"""torch.autograd wrappers of the forward operator (argument marshalling only).

``PatOperator.apply(p0, plan)`` returns the sensor data H p0 (shape
(nt, ns)); its backward is the exact adjoint H^T applied to the incoming
gradient, so ``torch.autograd`` computes grad f = H^T (H x - p) for the
least-squares term of the objective (equation Six of the paper) without
storing any forward time step: H is linear in p0.

The forward can run in time segments of ``ckpt_every`` samples through
``pat_forward_range``; the scheme's state at each segment boundary is kept
as a device snapshot (``ctx.checkpoints``), from which any segment can be
replayed bitwise (``replay_segment``).

``PatLeastSquares.apply(p0, target, plan)`` fuses H p0, the residual and the
float64 accumulation of 1/2 ||H p0 - target||^2 (returned as a float64
scalar tensor); its backward is H^T residual times the incoming gradient.
"""
from __future__ import annotations

from typing import List, Optional, Tuple

import torch

from . import Plan, residual_f64, residual_f64_batched

__all__ = ["PatOperator", "PatLeastSquares", "PatBatchLeastSquares", "forward_checkpointed", "replay_segment"]


def forward_checkpointed(plan: Plan, p0: torch.Tensor, every: int,
                         data: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, List[Tuple[int, torch.Tensor]]]:
    """H p0 in segments [0, k), [k, 2k), ...; returns the data and the list of
    (sample index, state snapshot) at every segment boundary."""
    if every < 1:
        raise ValueError("every must be >= 1")
    if data is None:
        data = torch.empty((plan.nt, plan.ns), device=p0.device, dtype=torch.float32)
    ckpts: List[Tuple[int, torch.Tensor]] = []
    state = torch.empty(plan.state_bytes, dtype=torch.uint8, device=p0.device)
    a = 0
    while a < plan.nt:
        b = min(plan.nt, a + every)
        plan.forward_range(p0 if a == 0 else None, data, a, b, state)
        if b < plan.nt:
            ckpts.append((b, state.clone()))
        a = b
    return data, ckpts


def replay_segment(plan: Plan, ckpts: List[Tuple[int, torch.Tensor]], p0: torch.Tensor, n_begin: int,
                   n_end: int) -> torch.Tensor:
    """Samples [n_begin, n_end) recomputed from the nearest earlier snapshot
    (or from p0); returns a (n_end - n_begin, ns) tensor."""
    start, snap = 0, None
    for n, s in ckpts:
        if n <= n_begin and n > start:
            start, snap = n, s
    data = torch.empty((plan.nt, plan.ns), device=p0.device, dtype=torch.float32)
    state = torch.empty(plan.state_bytes, dtype=torch.uint8, device=p0.device)
    if snap is not None:
        state.copy_(snap)
    plan.forward_range(p0 if start == 0 else None, data, start, n_end, state)
    return data[n_begin:n_end].clone()


class PatOperator(torch.autograd.Function):
    """data = H p0; backward: grad_p0 = H^T grad_data."""

    @staticmethod
    def forward(ctx, p0: torch.Tensor, plan: Plan, ckpt_every: int = 0):
        p0c = p0.detach().contiguous()
        if ckpt_every and ckpt_every < plan.nt:
            data, ckpts = forward_checkpointed(plan, p0c, ckpt_every)
        else:
            data, ckpts = plan.forward(p0c), []
        ctx.plan = plan
        ctx.checkpoints = ckpts
        return data

    @staticmethod
    def backward(ctx, grad_data: torch.Tensor):
        g = ctx.plan.adjoint(grad_data.detach().to(torch.float32).contiguous())
        return g, None, None


class PatLeastSquares(torch.autograd.Function):
    """f = 1/2 ||H p0 - target||^2 accumulated in float64; backward H^T r."""

    @staticmethod
    def forward(ctx, p0: torch.Tensor, target: torch.Tensor, plan: Plan, ckpt_every: int = 0):
        p0c = p0.detach().contiguous()
        if ckpt_every and ckpt_every < plan.nt:
            data, _ = forward_checkpointed(plan, p0c, ckpt_every)
        else:
            data = plan.forward(p0c)
        r, half = residual_f64(data, target.detach().contiguous())
        ctx.plan = plan
        ctx.save_for_backward(r)
        return torch.tensor(half, dtype=torch.float64, device=p0.device)

    @staticmethod
    def backward(ctx, grad_f: torch.Tensor):
        (r,) = ctx.saved_tensors
        g = ctx.plan.adjoint(r)
        if float(grad_f) != 1.0:
            g = g * grad_f.to(torch.float32)
        return g, None, None, None


class PatBatchLeastSquares(torch.autograd.Function):
    """Batched f = sum_i 1/2 ||H_i p0_i - target_i||^2 (float64 scalar) over
    the instances of a ``Batch``; the backward is the batched adjoint of the
    residuals: grad p0_i = H_i^T (H_i p0_i - target_i) times the incoming
    gradient.

    ``PatBatchLeastSquares.apply(batch, targets, *p0s)``; targets is a list of
    (nt_i, ns_i) float32 device tensors in the batch's plan order."""

    @staticmethod
    def forward(ctx, batch, targets, *p0s):
        datas = batch.forward([p.detach().contiguous() for p in p0s])
        # all residuals and the objective in one call that leaves them on the
        # device: the adjoint is queued behind them without a host round trip
        res, out = residual_f64_batched(datas, [t.detach().contiguous() for t in targets])
        ctx.batch = batch
        ctx.save_for_backward(*res)
        return out[-1].clone()

    @staticmethod
    def backward(ctx, grad_f):
        grads = ctx.batch.adjoint(list(ctx.saved_tensors))
        # scaled on the device (exact for the usual 1): reading grad_f on the
        # host would wait for the whole forward
        torch._foreach_mul_(grads, grad_f.to(torch.float32))
        return (None, None, *grads)
