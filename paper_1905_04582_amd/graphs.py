"""Whole leapfrog trajectories and HMC chains captured once as HIP graphs
and replayed.

The library's calls are asynchronous, allocate nothing and take every
quantity that may change between replays (sigma, the step size, the prior
precision) as device scalars, so one ``mds_leapfrog`` call -- n_steps + 1
sweep/finalize pairs and the two energy reductions -- can be captured on
torch's capture stream and replayed with a single launch.
"""
from __future__ import annotations

import torch

from . import api


class LeapfrogGraph:
    """A captured trajectory with its own static input/output buffers.

    After ``set_inputs(x, p, ...)`` and ``replay()``, ``x``/``p`` hold the end
    point, ``grad``/``loglik`` the gradient of log pi and L there, and
    ``energy_start``/``energy_end`` the Hamiltonian before and after.
    """

    def __init__(self, problem: "api.MDSProblem", n_steps: int, sigma: float, step: float,
                 prior: float | None = None, inv_mass: torch.Tensor | None = None,
                 cached_gradient: bool = False):
        dev = problem.device
        n, d = problem.n, problem.d
        f64 = dict(dtype=torch.float64, device=dev)
        self.problem = problem
        self.n_steps = int(n_steps)
        self.cached_gradient = bool(cached_gradient)
        self.x = torch.zeros((n, d), **f64)
        self.p = torch.zeros((n, d), **f64)
        self.grad = torch.zeros((n, d), **f64)
        self.loglik = torch.zeros((), **f64)
        self.energy_start = torch.zeros((), **f64)
        self.energy_end = torch.zeros((), **f64)
        self.sigma = torch.full((), float(sigma), **f64)
        self.step = torch.full((), float(step), **f64)
        self.prior = None if prior is None else torch.full((), float(prior), **f64)
        self.inv_mass = None if inv_mass is None else inv_mass.to(**f64).contiguous()

        # torch requires a warm-up on a side stream before capture
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            self._call(0)
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._call(self.n_steps)

    def _call(self, steps):
        self.problem.leapfrog(self.x, self.p, self.sigma, self.step, steps, self.grad,
                              self.loglik, cache_valid=self.cached_gradient,
                              inv_mass=self.inv_mass, prior=self.prior,
                              energy_start=self.energy_start, energy_end=self.energy_end)

    def set_inputs(self, x=None, p=None, sigma=None, step=None, prior=None, grad=None,
                   loglik=None):
        if x is not None:
            self.x.copy_(x)
        if p is not None:
            self.p.copy_(p)
        if sigma is not None:
            self.sigma.fill_(float(sigma))
        if step is not None:
            self.step.fill_(float(step))
        if prior is not None:
            if self.prior is None:
                raise ValueError("the graph was captured without a prior")
            self.prior.fill_(float(prior))
        if grad is not None:
            self.grad.copy_(grad)
        if loglik is not None:
            self.loglik.copy_(loglik)

    def replay(self):
        self.graph.replay()


class HMCChainGraph:
    """HMC transitions (momentum draw, leapfrog trajectory, Metropolis test,
    restore on rejection) captured once as a graph; each ``run(k)`` replays it
    k times, i.e. advances the chain by k * transitions_per_graph transitions
    without any host round trip.  The transition counter, the acceptance
    count and the last transition's statistics live in device tensors:
    ``iteration``, ``accepted``, ``stats`` (H_start, H_end, ln u, accepted).
    """

    def __init__(self, problem: "api.MDSProblem", x0, n_steps: int, sigma: float, step: float,
                 seed: int, prior: float | None = None, inv_mass: torch.Tensor | None = None,
                 transitions_per_graph: int = 1, first_iteration: int = 0):
        dev = problem.device
        n, d = problem.n, problem.d
        f64 = dict(dtype=torch.float64, device=dev)
        i64 = dict(dtype=torch.int64, device=dev)
        self.problem = problem
        self.n_steps = int(n_steps)
        self.seed = int(seed)
        self.per_graph = int(transitions_per_graph)
        self.x = torch.as_tensor(x0, **f64).clone().contiguous()
        self.p = torch.zeros((n, d), **f64)
        self.grad = torch.zeros((n, d), **f64)
        self.loglik = torch.zeros((), **f64)
        self.stats = torch.zeros(4, **f64)
        self.iteration = torch.full((1,), int(first_iteration), **i64)
        self.accepted = torch.zeros(1, **i64)
        self.sigma = torch.full((), float(sigma), **f64)
        self.step = torch.full((), float(step), **f64)
        self.prior = None if prior is None else torch.full((), float(prior), **f64)
        self.inv_mass = None if inv_mass is None else inv_mass.to(**f64).contiguous()

        # grad log pi and L at x0 (the captured transitions reuse the cache)
        problem.leapfrog(self.x, self.p, self.sigma, self.step, 0, self.grad, self.loglik,
                         inv_mass=self.inv_mass, prior=self.prior)
        saved = [t.clone() for t in (self.x, self.grad, self.loglik, self.iteration)]
        # torch requires a warm-up on a side stream before capture
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            self._transitions(1)
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._transitions(self.per_graph)
        # undo the warm-up transition
        for t, s in zip((self.x, self.grad, self.loglik, self.iteration), saved):
            t.copy_(s)
        self.accepted.zero_()
        torch.cuda.synchronize(dev)

    def _transitions(self, k):
        for _ in range(k):
            self.problem.hmc_step(self.x, self.p, self.sigma, self.step, self.n_steps, self.seed,
                                  self.iteration, self.grad, self.loglik, cache_valid=True,
                                  inv_mass=self.inv_mass, prior=self.prior, stats=self.stats,
                                  accepted_total=self.accepted)

    def run(self, replays: int = 1):
        for _ in range(int(replays)):
            self.graph.replay()
