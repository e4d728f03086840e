"""Transient problems: a sequence of related solves with a choice of initial
guess, and the training of the learned guess on the solver's own solutions.

Backward Euler for the heat equation (problems.heat_transient):
A u^m = u^{m-1} + dt f^m, m = 1 .. steps, every solve by the library's FP64
pipelined CG (Algorithm 2) to a relative residual tolerance.  Initial
guesses:
  "prev"    x0 = u^{m-1}                 (the method without a model)
  "extrap"  x0 = 2 u^{m-1} - u^{m-2}
  "learned" x0 = fk_net_guess(...)       (extrapolation corrected by the
                                          network, `passes` times, falling
                                          back to u^{m-1})
Vector work (b, the extrapolation, copies) runs in the library's kernels;
this module only orders the calls.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import fk
from . import problems as P

POLICIES = ("prev", "extrap", "learned")


@dataclass
class RunResult:
    policy: str
    iterations: np.ndarray   # CG iterations of each step
    seconds: float           # wall time of all steps (guess + solve)
    statuses: list

    @property
    def total_iterations(self) -> int:
        return int(self.iterations.sum())

    @property
    def solves_per_s(self) -> float:
        return len(self.iterations) / self.seconds


class Transient:
    """One transient problem resident on the device."""

    def __init__(self, n: int = 512, seed: int = 0, steps: int = 400, rtol: float = 1e-8,
                 unroll: int = 4, device: str = "cuda", method: str = "cg_pipelined"):
        """method: the CG schedule that solves each step ("cg_pipelined", two
        kernels per iteration, or "cg_pipelined_1k", one; same iterates)."""
        import torch

        A, u0, source = P.heat_transient(n, seed, steps)
        self.A = A
        self.n = n
        self.N = A.n
        self.steps = steps
        self.rtol = rtol
        self.M = fk.Matrix(A)
        self.u0 = torch.as_tensor(u0, device=device)
        # sources[m-1] = dt f^m
        self.sources = torch.empty((steps, A.n), dtype=torch.float64, device=device)
        for m in range(1, steps + 1):
            self.sources[m - 1].copy_(torch.as_tensor(source(m)))
        self.unroll = unroll
        self.method = method
        self.solver = fk.Solver(self.M, method=method, rtol=rtol, record_history=False,
                                unroll=unroll, small=False)
        self.device = device

    def run(self, policy: str, net: fk.Net | None = None, keep: bool = False,
            rtol: float | None = None, passes: int = 1) -> tuple[RunResult, object]:
        """All steps with one guess policy; returns the result and (keep=True)
        the solutions u^0 .. u^steps as a (steps+1, N) device tensor."""
        import torch

        if policy not in POLICIES:
            raise ValueError(policy)
        if policy == "learned" and net is None:
            raise ValueError("the learned policy needs a network")
        solver = self.solver
        if rtol is not None and rtol != self.rtol:
            solver = fk.Solver(self.M, method=self.method, rtol=rtol, record_history=False,
                               unroll=self.unroll, small=False)
        N = self.N
        traj = torch.empty((self.steps + 1, N), dtype=torch.float64, device=self.device) if keep else None
        bufs = [self.u0.clone(), self.u0.clone(), torch.empty_like(self.u0)]
        b = torch.empty_like(self.u0)
        if keep:
            traj[0].copy_(self.u0)
        prev, cur, nxt = bufs  # u^{m-2}, u^{m-1}, x
        iters, statuses = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for m in range(1, self.steps + 1):
            fk.axpby(1.0, cur, 1.0, self.sources[m - 1], b)
            if policy == "prev":
                fk.axpby(1.0, cur, 0.0, cur, nxt)
            elif policy == "extrap":
                fk.axpby(2.0, cur, -1.0, prev, nxt)
            else:
                net.guess(self.M, self.n, self.n, b, cur, prev, nxt, passes=passes)
            st = solver.solve(b, nxt)
            iters.append(solver.iterations())
            statuses.append(st)
            if keep:
                traj[m].copy_(nxt)
            prev, cur, nxt = cur, nxt, prev
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return RunResult(policy, np.array(iters), dt, statuses), traj

    def sample(self, traj, m: int, b_out):
        """Training sample predicting u^{m+1}: b^{m+1} = u^m + dt f^{m+1} into
        b_out; returns (u^m, u^{m-1}, u^{m+1}) views (u^{-1} = u^0)."""
        fk.axpby(1.0, traj[m], 1.0, self.sources[m], b_out)
        return traj[m], traj[max(m - 1, 0)], traj[m + 1]


# The learned guess used by the benchmark and the tests: a linear network of
# 4 layers, trained for 3000 Adam steps on the solver's own solutions for
# seeds 1-3 mixed with 30 % broadband pairs, applied in 4 passes.
RECIPE = {"layers": 4, "activation": "linear", "train_seeds": (1, 2, 3), "iters": 3000,
          "broadband_share": 0.3, "broadband_fields": 64, "passes": 4, "init_seed": 0}


def train_recipe(recipe: dict = RECIPE, n: int = 512, report_every: int = 0):
    """Generate the training data with the solver, train a network per the
    recipe; returns (net, losses, seconds for data, seconds for training)."""
    import torch

    t0 = time.perf_counter()
    data = generate(recipe["train_seeds"], n=n)
    bb = Broadband(data[0][0], recipe["broadband_fields"], seed=5)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net = fk.Net(recipe["layers"], P.net_init(recipe["layers"], recipe["init_seed"]),
                 activation=recipe["activation"])
    losses = train(net, data, recipe["iters"], report_every=report_every, broadband=bb,
                   broadband_share=recipe["broadband_share"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return net, losses, t1 - t0, t2 - t1


def generate(seeds, n: int = 512, steps: int = 400, rtol: float = 1e-12):
    """Training trajectories from the solver itself (extrapolated guesses,
    tight tolerance): list of (Transient, solutions)."""
    data = []
    for s in seeds:
        T = Transient(n, s, steps, rtol=rtol)
        _, traj = T.run("extrap", keep=True)
        data.append((T, traj))
    return data


class Broadband:
    """Synthetic pairs for the approximate inverse: fields e (white noise
    plus a smooth random field, from default_rng(seed)) with r = A e, so
    that later passes, whose residuals are not smooth, are in the training
    distribution.  A sample is (b = A e, u_m = u_{m-1} = 0, u_next = e)."""

    def __init__(self, T: "Transient", count: int = 32, seed: int = 0):
        import torch

        rng = np.random.default_rng(seed)
        n = T.n
        t = np.arange(n) / n
        self.T = T
        self.e = torch.empty((count, T.N), dtype=torch.float64, device=T.device)
        self.b = torch.empty_like(self.e)
        self.zero = torch.zeros(T.N, dtype=torch.float64, device=T.device)
        for k in range(count):
            white = rng.uniform(-1.0, 1.0, T.N)
            fx, fy, ph = rng.uniform(1, 40, 2), rng.uniform(1, 40, 2), rng.uniform(0, 2 * np.pi, 2)
            smooth = np.outer(np.sin(fy[0] * t + ph[0]), np.sin(fx[0] * t + ph[1])).ravel()
            e = white * 10.0 ** rng.uniform(-2, 0) + smooth
            self.e[k].copy_(torch.as_tensor(e))
            fk.spmv(T.M, self.e[k], self.b[k])

    def sample(self, k: int):
        return self.b[k], self.zero, self.zero, self.e[k]


def train(net: fk.Net, data, iters: int, lr: float = 2e-3, lr_final: float = 5e-4, seed: int = 0,
          report_every: int = 0, broadband: Broadband | None = None,
          broadband_share: float = 0.0) -> list[tuple[int, float]]:
    """Adam on samples (trajectory, step) drawn from default_rng(seed) (and,
    with probability broadband_share, synthetic pairs); the step size drops
    from lr to lr_final halfway.  Returns the reported losses."""
    import torch

    rng = np.random.default_rng(seed)
    b = None
    losses = []
    for it in range(iters):
        T, traj = data[int(rng.integers(len(data)))]
        m = int(rng.integers(0, T.steps))
        syn = broadband is not None and rng.uniform() < broadband_share
        if b is None or b.numel() != T.N:
            b = torch.empty(T.N, dtype=torch.float64, device=traj.device)
        if syn:
            bb, um, um1, un = broadband.sample(int(rng.integers(broadband.e.shape[0])))
            step = lr if it < iters // 2 else lr_final
            report = report_every > 0 and (it % report_every == 0 or it == iters - 1)
            loss = net.train_step(broadband.T.M, T.n, T.n, bb, um, um1, un, step, report=report)
            if report:
                losses.append((it, loss))
            continue
        um, um1, un = T.sample(traj, m, b)
        step = lr if it < iters // 2 else lr_final
        report = report_every > 0 and (it % report_every == 0 or it == iters - 1)
        loss = net.train_step(T.M, T.n, T.n, b, um, um1, un, step, report=report)
        if report:
            losses.append((it, loss))
    return losses
