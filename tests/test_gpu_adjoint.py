"""GPU step adjoints over a batch of uneven simulations against the
oracle's forward sensitivities and against central finite differences of
the GPU forward run."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_09435_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2507_09435_amd import mpm as M
    M.load()
    assert torch.cuda.is_available()
    c = M.mpm_create(0)
    yield c
    M.mpm_destroy(c)


def plastic_footing(n_y):
    """Footing reading used for gradients: cohesion 1 kPa, associated flow,
    0.1 mm pushes."""
    return W.gradient_reading(W.small_footing(n_y=n_y))


CASES = [(5, 2e7, 28.0), (6, 1e7, 32.0), (4, 5e6, 25.0)]
STEPS = [0, 1, 2, 3]


def _batch():
    return [plastic_footing(n) for n, _, _ in CASES]


def test_batched_adjoint_matches_oracle_sensitivity(ctx):
    from paper_2507_09435_amd import adjoint as AD
    sims = _batch()
    E = [c[1] for c in CASES]
    phi = [math.radians(c[2]) for c in CASES]
    print("[adjoint] batch forward", flush=True)
    dp = AD.make_batch(sims, E, phi)
    run = AD.forward(ctx, dp, sims, STEPS, tol=1e-12)
    R = run.reactions
    gR = 2.0 * (R - 0.9 * R)                       # loss sum_n (R_n - 0.9 R_n)^2 per sim
    theta = AD.backward(ctx, run, gR).cpu().numpy()
    for s, w in enumerate(sims):
        P = w.prob
        P.E, P.phi = E[s], phi[s]
        st = w.particles.copy()
        st.E = st.phi = None
        Ro, dRo, _ = O.simulate_sensitivity(P, st, [w.bc(k) for k in STEPS], w.footing_nodes(), 1, tol=1e-12)
        np.testing.assert_allclose(R[:, s], Ro, rtol=1e-9, atol=1e-9 * np.abs(Ro).max())
        ref = gR[:, s] @ dRo
        print(f"  sim {s}: dL/dE {theta[s, 0]:.6e} vs {ref[0]:.6e}; dL/dphi {theta[s, 1]:.6e} vs {ref[1]:.6e}",
              flush=True)
        np.testing.assert_allclose(theta[s], ref, rtol=1e-8, atol=1e-8 * np.abs(ref).max())


def test_adjoint_matches_gpu_central_fd(ctx):
    from paper_2507_09435_amd import adjoint as AD
    w = plastic_footing(6)
    E, phi = 1e7, math.radians(30.0)

    def loss_and_run(E_, phi_):
        dp = AD.make_batch([w], [E_], [phi_])
        run = AD.forward(ctx, dp, [w], STEPS, tol=1e-13)
        return float((run.reactions[:, 0] ** 2).sum()), run

    L0, run = loss_and_run(E, phi)
    th = AD.backward(ctx, run, 2.0 * run.reactions).cpu().numpy()[0]
    fd = []
    for k, d in enumerate([1e-6 * E, 1e-6]):
        args_p = (E + d, phi) if k == 0 else (E, phi + d)
        args_m = (E - d, phi) if k == 0 else (E, phi - d)
        fd.append((loss_and_run(*args_p)[0] - loss_and_run(*args_m)[0]) / (2 * d))
    print(f"[adjoint fd] {th} vs {fd}", flush=True)
    np.testing.assert_allclose(th, fd, rtol=1e-5)
