"""torch.autograd binding of the solver: T = BTESolve.apply(solver, tau, Q).

The forward pass runs the HIP source iteration to convergence with the given
relaxation times and keeps the angular field; the backward pass runs the
library's hand-written adjoint (transpose sweeps and the implicit-function
adjoint of the fixed point) and returns dJ/dtau_b and dJ/dQ_c. The gradient is
that of the converged discrete fixed point, not of the iterates.

If the solver has solved again or changed tau between this forward pass and
its backward pass (its ``generation`` moved), the stored state belongs to
another point: the backward pass then solves again at this pass's tau and Q
before the adjoint, so the gradient is always the one of this forward pass.
"""
from __future__ import annotations

import torch


class BTESolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, tau, Q, opts=None):
        opts = dict(opts or {})
        tau_np = tau.detach().to("cpu", torch.float64).numpy().copy()
        Qd = Q.detach().to(torch.float64).contiguous()
        T, _, rep = solver.solve(Qd, tau=tau_np, store_state=True, **opts)
        ctx.solver = solver
        ctx.opts = opts
        ctx.tau_np = tau_np
        ctx.Q = Qd
        ctx.generation = solver.generation
        ctx.tau_meta = (tau.device, tau.dtype)
        ctx.report = rep
        return T

    @staticmethod
    def backward(ctx, gT):
        s = ctx.solver
        if s.generation != ctx.generation:
            s.solve(ctx.Q, tau=ctx.tau_np, store_state=True, **ctx.opts)
        dtau, dQ, _ = s.adjoint(gT.detach().to(torch.float64).contiguous(), **ctx.opts)
        dev, dt = ctx.tau_meta
        return None, torch.as_tensor(dtau, device=dev, dtype=dt), dQ, None
