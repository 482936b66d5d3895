"""The Neo-Hookean law on the HIP path (Sec. 4.5's material) against the
oracle, and the stiffness identification by gradient descent over the step
adjoints: its gradient against central differences of the same GPU runs,
and the descent from a tenfold underestimate of E to the reference
stiffness."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_09435_amd import workloads as W

from gpu_common import row_errors, block_errors, compact_to_full, react_mask, rel_err, seeded_du

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2507_09435_amd import mpm as M
    M.load()
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    c = M.mpm_create(0)
    yield c
    M.mpm_destroy(c)


def _case(name):
    if name == "footing":
        from paper_2507_09435_amd import inverse as INV
        return INV.neo_hookean_footing(8, 1e7, 2), 1
    if name == "cube":
        w = W.make_c3(n=8, n_steps=1)
        w.prob.dp, w.prob.elastic = 0, 1
        return w, 0
    if name == "up":
        w = W.make_c4(n=8, n_steps=1, width_cells=4, dt=1.0)
        w.prob.elastic = 1
        return w, 1
    raise KeyError(name)


@pytest.mark.parametrize("name", ["footing", "cube", "up"])
def test_neohookean_residual_and_jacobian_parity(ctx, name):
    from paper_2507_09435_amd import mpm as M
    print(f"[nh] residual/jacobian case={name}", flush=True)
    w, step = _case(name)
    P, st = w.prob, w.particles
    dp = M.make_problem([(P, st)], [w.bc(step)], react_masks=[react_mask(w)])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    pat = O.pattern(P, st)
    du = seeded_du(P, pat, seed=61, amp=2e-2)
    dut = torch.from_numpy(du.reshape(-1)).cuda()
    rr = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    M.mpm_residual(ctx, dp, dut, None, rr)
    val = torch.zeros(nnzb * nd * nd, dtype=torch.float64, device="cuda")
    M.mpm_jacobian_bsr(ctx, dp, dut, val=val, raw=True)
    torch.cuda.synchronize()
    full = compact_to_full(P, pat, du)
    fint, fext = O.forces(P, st, full)
    ref = (fint - fext)[pat.active]
    scale = max(np.linalg.norm(ref), np.linalg.norm(fint[pat.active]), np.linalg.norm(fext[pat.active]))
    e = rel_err(rr.cpu().numpy().reshape(-1, nd), ref, scale)
    assert row_errors(rr.cpu().numpy(), ref, fint[pat.active], fext[pat.active]).max() <= 1e-10
    be = block_errors(val.cpu().numpy(), O.jacobian_bsr(P, st, full, pat)).max()
    print(f"  residual {e:.2e}, worst Jacobian block {be:.2e}", flush=True)
    assert e <= 1e-10 and be <= 1e-9


def test_neohookean_newton_step_and_update(ctx):
    from paper_2507_09435_amd import mpm as M
    w, step = _case("footing")
    P, st = w.prob, w.particles
    b0 = w.bc(0)
    d0, _, _ = O.newton(P, st, b0.mask, b0.value, tol=1e-13)
    st = O.update(P, st, d0)
    bc = w.bc(1)
    dp = M.make_problem([(P, st)], [bc], react_masks=[react_mask(w)])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    rep = M.mpm_newton_step(ctx, dp, du, tol=1e-13, commit=True, krylov_rtol=1e-13, krylov_method=2)
    torch.cuda.synchronize()
    assert rep["converged"]
    dof, orep, pat = O.newton(P, st, bc.mask, bc.value, tol=1e-13)
    got = du.cpu().numpy().reshape(-1, nd)
    e = rel_err(got, dof[pat.active])
    new = O.update(P, st, dof)
    be = dp.tensors["be"].cpu().numpy().reshape(4, -1)
    print(f"[nh] newton du rel err {e:.2e}; b^e after update max diff {np.abs(be - new.be).max():.2e}", flush=True)
    assert e <= 1e-10
    assert np.abs(be - new.be).max() <= 1e-11


def test_identification_gradient_and_descent(ctx):
    """Two footings (true E = 10 MPa and 30 MPa) identified at once from a
    tenfold underestimate: the adjoint gradient of the first iteration
    matches central differences of the GPU losses, and every sim's E ends
    within 0.2 % of its truth with the loss below 1e-6."""
    from paper_2507_09435_amd import inverse as INV
    E_true = [1e7, 3e7]
    E0 = [1e6, 3e6]
    sims = [INV.neo_hookean_footing(8, e, 4) for e in E0]
    opts = dict(tol=1e-12, krylov_rtol=1e-13, krylov_method=0)
    E, hist = INV.identify(ctx, sims, E_true, E0, lr=0.2, loss_tol=1e-6, max_iter=40, **opts)
    for k, (e, l) in enumerate(zip(hist.E, hist.loss)):
        print(f"[inverse] iteration {k}: E {np.array2string(e, precision=4)}  loss {np.array2string(l, precision=3)}",
              flush=True)
    assert all(abs(e / t - 1) < 2e-3 for e, t in zip(E, E_true)), E
    assert (hist.loss[-1] < 1e-6).all()
    # gradient check at the start: dL/dtheta by central differences of the GPU loss
    import torch as T
    from paper_2507_09435_amd import adjoint as AD
    curves = AD.ReactionCurves(ctx, sims, list(range(5)), **opts)
    phi = T.zeros(2, dtype=T.float64)
    s_ref = INV.slopes(curves(T.tensor(E_true, dtype=T.float64), phi), -2e-4)

    def loss(theta):
        with T.no_grad():
            return ((T.log(INV.slopes(curves(T.exp(theta), phi), -2e-4)) - T.log(s_ref)) ** 2).numpy()

    th0 = T.log(T.tensor(E0, dtype=T.float64))
    h = 1e-5
    fd = (loss(th0 + h) - loss(th0 - h)) / (2 * h)
    g = hist.grad[0]
    print(f"[inverse] dL/dtheta adjoint {g}  central differences {fd}", flush=True)
    assert np.all(np.abs(g - fd) <= 1e-5 * np.abs(fd) + 1e-10), (g, fd)
