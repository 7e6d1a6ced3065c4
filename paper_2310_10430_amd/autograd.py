"""torch.autograd front end of the discrete adjoint (biot_adjoint).

`pressure_misfit(logk, lam, mu, problem, sensors, p_obs)` returns the scalar
    J = sum_{n=1..N} sum_s (p^n(node_s) - p_obs[n-1, s])^2
of the backward-Euler trajectory (solved by the inverted iteration on the GPU)
for per-element log-permeability and Lame parameters, and its backward pass
calls the library's adjoint sweep.  A global lambda or mu is passed as an
expanded scalar; autograd then sums the per-element gradient.  Only argument
marshalling happens here: the forward solve, J, the adjoint solve, the
checkpoint replay and the gradient contraction all run in the HIP library.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from .solver import BiotSolver


class PressureMisfit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, logk, lam, mu, problem, sensors, p_obs, config):
        cfg = dict(config or {})
        rtol = float(cfg.pop("rtol", 1e-10))
        adj_rtol = float(cfg.pop("adjoint_rtol", rtol))
        max_sweeps = int(cfg.pop("max_sweeps", 4000))
        device = cfg.pop("device", "cuda:0")
        sensors = np.asarray(sensors, dtype=np.int32)
        p_obs = np.asarray(p_obs, dtype=np.float64)
        host = lambda t: t.detach().to("cpu", torch.float64).numpy()
        pb = dataclasses.replace(problem, perm=np.exp(host(logk)))
        solver = BiotSolver(pb, device=device, lame=(host(lam), host(mu)), adjoint=True,
                            max_sensors=max(int(sensors.size), 1), **cfg)
        solver.solve_to_tol(rtol, max_sweeps=max_sweeps)
        J = solver.objective(sensors, p_obs)
        ctx.solver = solver
        ctx.args = (sensors, p_obs, adj_rtol, max_sweeps)
        ctx.devices = (logk.device, lam.device, mu.device)
        return torch.tensor(J, dtype=torch.float64, device=logk.device)

    @staticmethod
    def backward(ctx, gJ):
        sensors, p_obs, rtol, max_sweeps = ctx.args
        solver = ctx.solver
        try:
            out = solver.adjoint(sensors, p_obs, rtol=rtol, max_sweeps=max_sweeps)
            g = [out["grad_logk"], out["grad_lambda"], out["grad_mu"]]
            scale = gJ.to(solver.device, torch.float64)
            grads = [(gi * scale).to(dev) for gi, dev in zip(g, ctx.devices)]
        finally:
            solver.close()
            ctx.solver = None
        return grads[0], grads[1], grads[2], None, None, None, None


def pressure_misfit(logk: torch.Tensor, lam: torch.Tensor, mu: torch.Tensor, problem, sensors,
                    p_obs, **config) -> torch.Tensor:
    """J(log K, lambda, mu); extra keywords go to BiotSolver (schedule, depth,
    precision, ckpt_stride, ...) plus rtol, adjoint_rtol, max_sweeps, device."""
    return PressureMisfit.apply(logk, lam, mu, problem, sensors, p_obs, config)
