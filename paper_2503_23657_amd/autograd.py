"""torch.autograd binding of the solver: T = BTESolve.apply(solver, tau, Q).

The forward pass runs the HIP source iteration to convergence and keeps the
angular field; the backward pass runs the library's hand-written adjoint
(transpose sweeps and the implicit-function adjoint of the fixed point) and
returns dJ/dtau_b and dJ/dQ_c. The gradient is that of the converged discrete
fixed point, not of the iterates.
"""
from __future__ import annotations

import numpy as np
import torch


class BTESolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, tau, Q, opts=None):
        opts = dict(opts or {})
        tau_np = tau.detach().to("cpu", torch.float64).numpy()
        if getattr(solver, "_tau_set", None) is None or not np.array_equal(solver._tau_set, tau_np):
            solver.set_tau(tau_np)
            solver._tau_set = tau_np.copy()
        T, _, rep = solver.solve(Q.detach().to(torch.float64).contiguous(), store_state=True, **opts)
        ctx.solver = solver
        ctx.opts = opts
        ctx.tau_meta = (tau.device, tau.dtype)
        ctx.report = rep
        return T

    @staticmethod
    def backward(ctx, gT):
        dtau, dQ, _ = ctx.solver.adjoint(gT.detach().to(torch.float64).contiguous(), **ctx.opts)
        dev, dt = ctx.tau_meta
        return None, torch.as_tensor(dtau, device=dev, dtype=dt), dQ, None
