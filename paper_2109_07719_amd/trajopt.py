"""Gradient-based trajectory optimisation through the differentiable rollout.

The control sequence tau[T] of every system is a torch parameter; the loss
is ||end-effector(q^T) - target||^2 + w ||tau||^2, optimised with Adam.  One
iteration = rollout (forward kernel with checkpoints) -> torch forward
kinematics and loss -> loss.backward() (torch FK backward gives dL/dq^T,
the adjoint kernel gives dL/dtau) -> Adam step.  This is the motion-control
use of the gradients (Sec. 6.3: optimising a torque sequence towards a
target), on batched synthetic chains.
"""
from __future__ import annotations

import numpy as np
import torch

from .fk import LinkPoints
from .sim import Sim, rollout


class TrajOpt:
    def __init__(self, batch, targets, ee_links, ee_points, lr=1e-2, tau_weight=1e-4, K=1,
                 dtype=torch.float32, device="cuda"):
        self.b = batch
        self.sim = Sim(batch.systems, batch.gravity, dtype=dtype, device=device)
        self.fk = LinkPoints(batch.systems, ee_links, ee_points, dtype=dtype, device=device)
        f = lambda x: torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=device)
        self.q0, self.qd0 = f(batch.q0), f(batch.qd0)
        self.target = f(targets)
        self.tau = torch.nn.Parameter(f(batch.tau))
        self.opt = torch.optim.Adam([self.tau], lr=lr)
        self.w, self.K, self.dt = tau_weight, K, batch.dt

    def loss(self):
        qT, _ = rollout(self.sim, self.q0, self.qd0, self.tau, self.dt, K=self.K)
        ee = self.fk(qT)
        per_sys = ((ee - self.target) ** 2).sum(-1)
        return per_sys.sum() + self.w * (self.tau ** 2).sum(), per_sys

    def step(self):
        self.opt.zero_grad(set_to_none=False)
        L, per_sys = self.loss()
        L.backward()
        self.opt.step()
        return L.detach(), per_sys.detach()


def chains_problem(n_systems=2048, T=1000):
    """Chains of 5-50 links (seeds 4000+i), q0 = qd0 = 0, tau = 0; the
    end-effector is the point (0.5, 0, 0) of the last link; targets are the
    end-effector positions of random configurations q* ~ U(-pi, pi)^n."""
    from . import synth
    b = synth.round_to_f32(synth.workload("chains_2048", n_systems=n_systems, T=T))
    qstar = synth.chains_targets(n_systems)
    fk = LinkPoints(b.systems, [s.n - 1 for s in b.systems], np.tile([0.5, 0.0, 0.0], (n_systems, 1)),
                    dtype=torch.float64, device="cpu")
    targets = fk(torch.tensor(np.concatenate(qstar), dtype=torch.float64)).numpy()
    return b, targets
