"""Batched forward runs with step checkpoints and their adjoint.

Forward: every load step of a batch of simulations is one Newton solve
through the C ABI; the state at the start of each step (x, F, b^e) and the
converged increment are kept on the device.  Backward: the steps are
revisited in reverse, each one re-binned from its checkpoint and handed to
mpm_adjoint_step (one transposed solve per step), which returns the state
adjoint of the step start and the step's contribution to dL/d(E, phi) of
every simulation.  This is the gradient of the paper's inverse analysis
(Sec. 4.5) without a tape over Newton iterations.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import mpm as M


def react_mask(w):
    m = np.zeros((w.prob.n_nodes, w.prob.ndof), dtype=np.uint8)
    if w.footing is not None:
        m[w.footing_nodes(), w.footing[1]] = 1
    return m


@dataclass
class Run:
    dp: M.DeviceProblem
    sims: list
    steps: list
    reactions: np.ndarray          # [n_steps][nsim]
    checkpoints: list              # per step: (x, F, be) device clones at the step start
    increments: list               # per step: converged compact du (device)
    newton_iters: list
    krylov_iters: list
    newton_rel: list               # per step: largest ||r||/||r_0|| over sims at the accepted iterate


def make_batch(sims, E, phi):
    """Device problem of a batch; E, phi per sim (per-particle arrays)."""
    for w, e, f in zip(sims, E, phi):
        w.particles.E = np.full(w.particles.np, float(e))
        w.particles.phi = np.full(w.particles.np, float(f))
    return M.make_problem([(w.prob, w.particles) for w in sims], [w.bc(0) for w in sims],
                          react_masks=[react_mask(w) for w in sims])


def set_params(dp, sims, E, phi):
    import torch
    Ep = np.concatenate([np.full(w.particles.np, float(e)) for w, e in zip(sims, E)])
    Pp = np.concatenate([np.full(w.particles.np, float(f)) for w, f in zip(sims, phi)])
    dp.tensors["E"].copy_(torch.from_numpy(Ep))
    dp.tensors["phi"].copy_(torch.from_numpy(Pp))


def forward(ctx, dp, sims, steps, tol=1e-10, krylov_rtol=1e-12, max_iter=25, line_search=0, krylov_method=0,
            stall_factor=1e3, progress=None):
    """Run the load steps of a batch, keeping checkpoints; progress(step,
    report) is called after each step when given.  stall_factor = 0 makes
    every step reach ||r|| <= tol ||r_0|| (no early stop at the round-off
    floor), which the adjoint's r = 0 assumption and finite differences of
    the reactions want; each step's reached ratio is kept in newton_rel."""
    import torch
    T = dp.tensors
    R, cps, dus, nit, kit, rel = [], [], [], [], [], []
    for step in steps:
        M.set_bc(dp, [w.bc(step) for w in sims])
        cps.append((T["x"].clone(), T["F"].clone(), T["be"].clone()))
        n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
        du = torch.zeros(n_row * nd, dtype=torch.float64, device=T["x"].device)
        rep = M.mpm_newton_step(ctx, dp, du, tol=tol, max_iter=max_iter, commit=True, krylov_rtol=krylov_rtol,
                                line_search=line_search, krylov_method=krylov_method, stall_factor=stall_factor,
                                raise_on_fail=False)
        if rep["status"] != M.MPM_OK:
            bad = [(s, rep["sim_iters"][s], rep["sim_rel"][s]) for s in range(dp.nsim) if not rep["sim_converged"][s]]
            raise M.MPMError(rep["status"], f"load step {step}: {M.STATUS_NAMES.get(rep['status'], rep['status'])}; "
                                            f"sims not converged (sim, iterations, ||r||/||r0||): {bad[:8]}")
        R.append(rep["sim_reaction"])
        rel.append(max(rep["sim_rel"]) if rep["sim_rel"] else 0.0)
        dus.append(du)
        nit.append(rep["iters"])
        if progress is not None:
            progress(step, rep)
        kit.append(rep["krylov_iters"])
    return Run(dp, sims, list(steps), np.array(R), cps, dus, nit, kit, rel)


def backward(ctx, run: Run, react_bar, krylov_rtol=1e-12, progress=None):
    """dL/d(E, phi) per sim given dL/dR (array [n_steps][nsim]);
    progress(step, krylov_iters) is called after each step when given."""
    import torch
    dp = run.dp
    T = dp.tensors
    np_ = T["vol0"].shape[0]
    theta = torch.zeros(dp.nsim * 2, dtype=torch.float64, device=T["x"].device)
    step_theta = torch.zeros_like(theta)
    sbar = None
    for k in range(len(run.steps) - 1, -1, -1):
        x, F, be = run.checkpoints[k]
        T["x"].copy_(x)
        T["F"].copy_(F)
        T["be"].copy_(be)
        M.set_bc(dp, [w.bc(run.steps[k]) for w in run.sims])
        M.mpm_prepare(ctx, dp)
        sbar_n = torch.empty(10 * np_, dtype=torch.float64, device=T["x"].device)
        kit = M.mpm_adjoint_step(ctx, dp, run.increments[k], react_bar[k], sbar, sbar_n, step_theta, krylov_rtol)
        if progress is not None:
            progress(run.steps[k], kit)
        theta += step_theta
        sbar = sbar_n
    return theta.reshape(dp.nsim, 2)


class ReactionCurves:
    """torch.autograd.Function over a batch: (E, phi) per sim -> reactions
    [n_steps][nsim]; backward runs the step adjoints."""

    def __init__(self, ctx, sims, steps, **opts):
        self.ctx, self.sims, self.steps, self.opts = ctx, sims, steps, opts
        self.fn = self._make_fn()

    def _make_fn(self):
        import torch
        outer = self

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(fctx, E, phi):
                e, f = E.detach().cpu().numpy(), phi.detach().cpu().numpy()
                for w in outer.sims:
                    w.particles = w.particles.copy()
                dp = make_batch(outer.sims, e, f)
                fopts = {k: v for k, v in outer.opts.items() if k != "adjoint_progress"}
                run = forward(outer.ctx, dp, outer.sims, outer.steps, **fopts)
                fctx.run = run
                outer.last_run = run
                return torch.from_numpy(run.reactions.copy()).to(E.device)

            @staticmethod
            def backward(fctx, gR):
                th = backward(outer.ctx, fctx.run, gR.detach().cpu().numpy(),
                              krylov_rtol=outer.opts.get("krylov_rtol", 1e-12),
                              progress=outer.opts.get("adjoint_progress"))
                return th[:, 0].to(gR.device), th[:, 1].to(gR.device)

        return _F

    def __call__(self, E, phi):
        return self.fn.apply(E, phi)
