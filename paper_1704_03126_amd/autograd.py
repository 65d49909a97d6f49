"""torch.autograd binding of the flow rate and its discrete adjoint.

``DVMFlowRate.apply(delta, alpha, solver, instance)`` returns the flow rate Q
of Sec. III for the per-cell rarefaction field ``delta`` (a tensor of the
instance's grid shape, or a 0-d tensor for a uniform value) and the
accommodation coefficient ``alpha`` (0-d tensor); its backward calls
``dvm_grad`` (the discrete adjoint of the library) for dQ/d delta and
dQ/d alpha.  The solve itself runs in the library's HIP kernels; torch only
carries the values and the graph.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dvm as _dvm


class DVMFlowRate(torch.autograd.Function):

    @staticmethod
    def forward(ctx, delta: torch.Tensor, alpha: torch.Tensor, solver: "_dvm.Solver", instance: int = 0):
        d = delta.detach().to("cpu", torch.float64).numpy()
        a = float(alpha.detach().cpu())
        solver.solve(instance, d if d.ndim else float(d), a)
        Q, _ = solver.flow_rate(instance)
        ctx.solver, ctx.instance, ctx.epoch = solver, instance, solver.epoch
        ctx.delta_np, ctx.alpha = d, a
        ctx.delta_meta = (delta.shape, delta.dtype, delta.device)
        ctx.alpha_meta = (alpha.dtype, alpha.device)
        return torch.tensor(Q, dtype=torch.float64, device=delta.device)

    @staticmethod
    def backward(ctx, gQ: torch.Tensor):
        s = ctx.solver
        if s.epoch != ctx.epoch:
            # the solver was used since the forward pass: restore its state
            d = ctx.delta_np
            s.solve(ctx.instance, d if d.ndim else float(d), ctx.alpha)
        gd, ga = s.grad(ctx.instance)
        shape, dtype, device = ctx.delta_meta
        g = float(gQ.detach().cpu())
        if len(shape) == 0:
            gdelta = torch.tensor(float(gd.sum()) * g, dtype=dtype, device=device)
        else:
            gdelta = torch.from_numpy(np.ascontiguousarray(gd) * g).to(device=device, dtype=dtype)
        galpha = torch.tensor(ga * g, dtype=ctx.alpha_meta[0], device=ctx.alpha_meta[1])
        return gdelta, galpha, None, None


def flow_rate(solver: "_dvm.Solver", delta, alpha=1.0, instance: int = 0) -> torch.Tensor:
    """Differentiable flow rate of one instance (see DVMFlowRate)."""
    if not torch.is_tensor(delta):
        delta = torch.tensor(delta, dtype=torch.float64)
    if not torch.is_tensor(alpha):
        alpha = torch.tensor(float(alpha), dtype=torch.float64)
    return DVMFlowRate.apply(delta, alpha, solver, instance)
