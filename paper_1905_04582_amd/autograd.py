"""Reverse-mode differentiation of the MDS log-likelihood for torch.

``mds_log_likelihood(x, log_sigma, problem)`` returns the log-likelihood L of
Eq. (2) as a 0-d float64 tensor that torch can differentiate with respect to
the latent locations X (N x D, float32 or float64) and to ln(sigma).

Forward runs the log-likelihood-only sweep (``mds_loglik``).  Backward runs
the gradient sweep once (``mds_gradient``) with the upstream gradient passed
as a device scalar, so the kernels return dL/dX and dL/d(ln sigma) already
multiplied by it: no host synchronisation, no extra arithmetic in torch.  A
float32 X is promoted to float64 for the kernels and its gradient is returned
in float32.
"""
from __future__ import annotations

import torch

from . import api


class MDSLogLikelihood(torch.autograd.Function):

    @staticmethod
    def forward(ctx, x, log_sigma, problem):
        if x.dim() != 2 or x.shape != (problem.n, problem.d):
            raise ValueError(f"x must be {problem.n} x {problem.d}")
        x64 = x.detach().to(torch.float64).contiguous()
        sigma = torch.exp(log_sigma.detach().to(torch.float64)).reshape(())
        out = problem.loglik(x64, sigma)
        ctx.problem = problem
        ctx.x_dtype = x.dtype
        ctx.ls_dtype = log_sigma.dtype
        ctx.save_for_backward(x64, sigma)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        x64, sigma = ctx.saved_tensors
        problem = ctx.problem
        need_x, need_s = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_x or need_s):
            return None, None, None
        scale = grad_out.detach().to(torch.float64).reshape(()).contiguous()
        dls = torch.empty((), dtype=torch.float64, device=x64.device)
        g, _, _ = problem.gradient(x64, sigma, scale=scale, want_loglik=False,
                                   want_dsigma=False, dlogsigma=dls)
        gx = g.to(ctx.x_dtype) if need_x else None
        gs = dls.to(ctx.ls_dtype) if need_s else None
        return gx, gs, None


def mds_log_likelihood(x: torch.Tensor, log_sigma: torch.Tensor,
                       problem: "api.MDSProblem") -> torch.Tensor:
    """Differentiable L(X, sigma) of Eq. (2) for a prepared problem."""
    if not isinstance(log_sigma, torch.Tensor):
        log_sigma = torch.tensor(float(log_sigma), dtype=torch.float64, device=x.device)
    return MDSLogLikelihood.apply(x, log_sigma, problem)


def map_ascent(problem, x0, log_sigma0, steps: int = 10, lr_x: float = 1e-4,
               lr_s: float = 1e-6):
    """Plain gradient ascent on (X, ln sigma) through the autograd Function;
    returns (x, log_sigma, [L per step])."""
    x = x0.detach().clone().requires_grad_(True)
    ls = torch.as_tensor(log_sigma0, dtype=torch.float64, device=x0.device).detach().clone()
    ls.requires_grad_(True)
    trace = []
    for _ in range(steps):
        L = mds_log_likelihood(x, ls, problem)
        x.grad = None
        ls.grad = None
        L.backward()
        with torch.no_grad():
            x += lr_x * x.grad
            ls += lr_s * ls.grad
        trace.append(L.detach())
    return x.detach(), ls.detach(), torch.stack(trace)
