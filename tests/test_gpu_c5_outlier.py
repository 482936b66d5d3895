"""The batched-set sim whose central-difference gradient departs most from
the adjoint (sim 41, 81,608 particles, 1.4e-4 relative over an 11-step
horizon) against the oracle's forward sensitivity of the same steps
(tests/golden/c5_sim41_oracle.json, written by make_c5_sim41.py from the
oracle alone): the GPU reaction curve and the adjoint gradient of the
squared misfit both agree with it, so the departure is on the
finite-difference side (Sec. 4.5: gradients through plasticity).  The
friction gradient of sim 12, the other outlier, is checked against central
differences taken with a step large enough to clear the Newton stopping
noise."""
import json
import os

import numpy as np
import pytest

from paper_2507_09435_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c5_sim41_oracle.json")


@pytest.fixture(scope="module")
def ctx():
    from paper_2507_09435_amd import mpm as M
    M.load()
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    c = M.mpm_create(0)
    yield c
    M.mpm_destroy(c)


def test_outlier_sim_adjoint_matches_oracle_sensitivity(ctx):
    from paper_2507_09435_amd import adjoint as AD
    g = json.load(open(GOLDEN))
    sims, targets = W.make_c5(nsim=64, n_steps=30)
    w = sims[g["sim"]]
    assert w.particles.np == g["particles"]
    print(f"[c5-outlier] sim {g['sim']}, {w.particles.np} particles, {g['steps']} load steps", flush=True)
    opts = dict(tol=1e-12, stall_factor=100.0, krylov_rtol=1e-12, max_iter=50, krylov_method=2, line_search=4)
    curves = AD.ReactionCurves(ctx, [w], list(range(g["steps"])), **opts)
    E = torch.tensor([g["E"]], dtype=torch.float64, requires_grad=True)
    phi = torch.tensor([g["phi"]], dtype=torch.float64, requires_grad=True)
    R = curves(E, phi)
    Rg = R.detach().numpy()[:, 0]
    Ro, Rt = np.asarray(g["R"]), np.asarray(g["Rt"])
    eR = np.abs(Rg - Ro).max() / np.abs(Ro).max()
    loss = ((R[:, 0] - torch.from_numpy(Rt)) ** 2).sum()
    loss.backward()
    gE, gphi = float(E.grad[0]), float(phi.grad[0])
    eE = abs(gE - g["dL_dE"]) / abs(g["dL_dE"])
    ephi = abs(gphi - g["dL_dphi"]) / abs(g["dL_dphi"])
    print(f"  reaction curve {eR:.2e}; dL/dE {gE:.12g} (oracle {g['dL_dE']:.12g}, {eE:.1e}); "
          f"dL/dphi {gphi:.12g} (oracle {g['dL_dphi']:.12g}, {ephi:.1e})", flush=True)
    assert eR <= 1e-9
    assert eE <= 1e-8 and ephi <= 1e-8


def test_friction_gradient_against_central_differences_of_a_suitable_step(ctx):
    """Sim 12 of the batched set (177,608 particles): its friction gradient
    departs from central differences with a 1e-5 rad step by about 2e-5.
    The departure shrinks as the step grows (3e-4 at 1e-6 rad, 5e-6 at
    1e-4, 1e-7 at 3e-4), as a loss carrying a few 1e-9 of Newton stopping
    noise, divided by the step, would; at a 3e-4 rad step the difference
    quotient agrees with the adjoint within 1e-5 (Sec. 4.5: gradients of
    the reaction misfit)."""
    from paper_2507_09435_amd import adjoint as AD
    sims, targets = W.make_c5(nsim=64, n_steps=30)
    w = sims[12]
    print(f"[c5-fd] sim 12, {w.particles.np} particles, 11 load steps", flush=True)
    opts = dict(tol=1e-12, stall_factor=100.0, krylov_rtol=1e-12, max_iter=50, krylov_method=2, line_search=4)
    curves = AD.ReactionCurves(ctx, [w], list(range(11)), **opts)
    E0 = torch.tensor([float(w.particles.E[0])], dtype=torch.float64)
    phi0 = torch.tensor([float(w.particles.phi[0])], dtype=torch.float64)
    with torch.no_grad():
        Rt = curves(torch.tensor([targets[12][0]], dtype=torch.float64),
                    torch.tensor([targets[12][1]], dtype=torch.float64))
    E = E0.clone().requires_grad_(True)
    phi = phi0.clone().requires_grad_(True)
    ((curves(E, phi) - Rt) ** 2).sum().backward()
    gE, gphi = float(E.grad[0]), float(phi.grad[0])

    def loss(Ev, pv):
        with torch.no_grad():
            return float(((curves(Ev, pv) - Rt) ** 2).sum())

    d = 3e-4
    fd_phi = (loss(E0, phi0 + d) - loss(E0, phi0 - d)) / (2 * d)
    dE = 1e-5
    fd_E = (loss(E0 * (1 + dE), phi0) - loss(E0 * (1 - dE), phi0)) / (2 * dE * float(E0[0]))
    ephi, eE = abs(fd_phi - gphi) / abs(gphi), abs(fd_E - gE) / abs(gE)
    print(f"  dL/dphi adjoint {gphi:.12g}, central difference ({d:g} rad) {fd_phi:.12g}: {ephi:.1e}; "
          f"dL/dE adjoint {gE:.12g}, central difference ({dE:g} relative) {fd_E:.12g}: {eE:.1e}", flush=True)
    assert ephi <= 1e-5 and eE <= 1e-5
