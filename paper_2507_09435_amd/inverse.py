"""Ground stiffness identification by gradient descent (Sec. 4.5).

A rigid footing is pushed into Neo-Hookean ground over a number of load
steps; the loss compares the slope of the simulated force-displacement curve
with the slope of a reference response, and gradient descent with learning
rate 0.2 updates the stiffness until the loss falls below a threshold.  The
gradient comes from the step adjoints (one transposed solve per converged
step, `adjoint.ReactionCurves`), not from a tape over the Newton iterations.

Readings of what the paper leaves open (the slope, the parameter scale of
the learning rate) are fixed here: the slope is the least-squares slope of
reaction against footing displacement over the pushes, the parameter is
theta = ln E and the loss is (ln s - ln s*)^2, so that the rate 0.2 is
dimensionless.  Every simulation of a batch is identified at once (each has
its own E, target slope and loss; the adjoints of the batch are independent).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import adjoint as AD
from . import workloads as W


def neo_hookean_footing(n_y: int, E: float, n_steps: int, push: float = -2e-4, nu: float = 0.3) -> W.Workload:
    """The plane-strain footing geometry on Neo-Hookean ground (no
    plasticity): geostatic step 0, then n_steps pushes of `push` metres."""
    w = W.footing_2d(n_y, E, 30.0, n_steps, f"nh{n_y}", nu=nu)
    w.prob.dp = 0
    w.prob.elastic = 1
    w.footing = (w.footing[0], w.footing[1], w.footing[2], push)
    return w


def slopes(R: "torch.Tensor", push: float):
    """Least-squares slope of reaction against footing displacement over the
    push steps (rows 1.. of R [steps][nsim]; row 0 is the geostatic step)."""
    import torch
    n = R.shape[0] - 1
    d = torch.arange(1, n + 1, dtype=R.dtype, device=R.device) * abs(push)
    dc = d - d.mean()
    Rp = R[1:]
    return (dc[:, None] * (Rp - Rp.mean(dim=0, keepdim=True))).sum(dim=0) / (dc * dc).sum()


@dataclass
class History:
    E: list = field(default_factory=list)       # per iteration: E per sim
    loss: list = field(default_factory=list)    # per iteration: loss per sim
    grad: list = field(default_factory=list)    # per iteration: dL/dtheta per sim


def identify(ctx, sims, E_true, E0, lr: float = 0.2, loss_tol: float = 1e-6, max_iter: int = 30,
             push: float = -2e-4, **opts):
    """Gradient descent on theta = ln E for every sim of the batch until each
    loss (ln s - ln s*)^2 is below loss_tol; opts go to the forward and
    adjoint runs (Newton and Krylov tolerances).  Returns (E, History)."""
    import torch
    steps = list(range(0, sims[0].n_steps + 1))
    phi = torch.zeros(len(sims), dtype=torch.float64)
    curves = AD.ReactionCurves(ctx, sims, steps, **opts)
    with torch.no_grad():
        s_ref = slopes(curves(torch.tensor(E_true, dtype=torch.float64), phi), push)
    theta = torch.log(torch.tensor(E0, dtype=torch.float64))
    hist = History()
    for _ in range(max_iter + 1):
        th = theta.clone().requires_grad_(True)
        R = curves(torch.exp(th), phi)
        loss = (torch.log(slopes(R, push)) - torch.log(s_ref)) ** 2
        hist.E.append(torch.exp(theta).numpy().copy())
        hist.loss.append(loss.detach().numpy().copy())
        if bool((loss < loss_tol).all()):
            hist.grad.append(np.zeros(len(sims)))
            break
        loss.sum().backward()
        g = th.grad.detach()
        hist.grad.append(g.numpy().copy())
        done = loss.detach() < loss_tol
        theta = theta - lr * torch.where(done, torch.zeros_like(g), g)
    return torch.exp(theta).numpy(), hist
