"""Displacement misfit gradients through ``torch.autograd``.

``SensorDisplacement.apply(k, A, problem)`` runs the Euler-Cromer problem from its
initial state with slot stiffness ``k`` (nnz) and body-force magnitude ``A`` and returns
the displacement of the sensor nodes after ``problem.nsteps`` steps (m x 3).  Its
backward calls the library's reverse pass (break schedule of the forward run frozen,
checkpoints every ``problem.ckpt_every`` steps) on that forward run's recording; a
backward after another forward on the same simulation raises instead of returning the
later run's gradient.  Torch only carries the tensors: the
forward and reverse passes run in the HIP library.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch


@dataclass
class AdjointProblem:
    """A single-instance Euler-Cromer problem set up on ``sim`` (family, material, BCs)."""
    sim: object                    # paper_2105_04150_amd.Simulation
    b_hat: Optional[np.ndarray]    # n x 3 body-force direction (None: no body force)
    sensors: np.ndarray            # m user node ids
    nsteps: int
    ckpt_every: int = 100
    broken0: Optional[np.ndarray] = None   # initial broken set (nnz, e.g. a notch)

    def reset(self, k: np.ndarray, A: float) -> None:
        sim = self.sim
        n, nnz = sim.size()
        sim.set_bond_stiffness(k)
        if self.b_hat is not None:
            sim.set_body_force(self.b_hat, A)
        z = np.zeros((n, 3))
        br = np.zeros(nnz, dtype=np.uint8) if self.broken0 is None else self.broken0
        sim.set_state(u=z, v=z, a=z, broken=br)
        sim.set_step(0)


class SensorDisplacement(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k: torch.Tensor, A: torch.Tensor, problem: AdjointProblem):
        kk = k.detach().to("cpu", torch.float64).numpy()
        problem.reset(kk, float(A))
        ctx.recording = problem.sim.adj_forward(problem.nsteps, problem.ckpt_every)
        u = problem.sim.u()[problem.sensors]
        ctx.problem = problem
        return torch.from_numpy(u).to(k.device)

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        g = grad_u.detach().to("cpu", torch.float64).numpy()
        # the library refuses (PdmiError, PD_ESTATE) if the problem's simulation has
        # recorded another forward run since this one: its tape no longer holds this run
        gk, gA = ctx.problem.sim.adj_backward(ctx.problem.sensors, g, ctx.recording)
        dev = grad_u.device
        return torch.from_numpy(gk).to(dev), torch.tensor(gA, dtype=torch.float64, device=dev), None


def sensor_displacement(k: torch.Tensor, A: torch.Tensor, problem: AdjointProblem) -> torch.Tensor:
    return SensorDisplacement.apply(k, A, problem)
