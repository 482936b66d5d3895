"""Multi-step load paths of the configurations on the HIP path against the
oracle (Sec. 2.2: the load-step Newton loop; Sec. 4.4: consolidation).
Both sides run the same load steps from their own states; every step's
Newton increment is compared, and the oracle's residual at the GPU's
increment certifies each step.

* the u-p consolidation on a column of its 64-cell height copy, 8 cells wide
  (the consolidation is one-dimensional: rollers at the sides), all 100
  steps of dt = 1 s, with the GPU pore pressures against Terzaghi's series
  at t = 10, 20, 50 and 100 s;
* the 3-D footing cube on a 12^3 grid and the plane-strain footing at full
  size (256 x 128 cells), geostatic step then footing pushes, both in the
  converging reading of the footing path (1 kPa cohesion, associated flow,
  0.1 mm pushes; with c = 0 and psi = 0 the path is ill-posed for Newton)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_09435_amd import workloads as W

from gpu_common import compact_to_full, react_mask, rel_err

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


def _gpu_step(ctx, w, st, step, tol, method, sub=None):
    """One committed GPU load step from state st; returns (du compact, new
    state, report)."""
    from paper_2507_09435_amd import mpm as M
    P = w.prob
    dp = M.make_problem([(P, st)], [w.bc(step)], react_masks=[react_mask(w)])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    rep = M.mpm_newton_step(ctx, dp, du, tol=tol, max_iter=25, commit=True, krylov_rtol=1e-13, krylov_method=method)
    torch.cuda.synchronize()
    assert rep["converged"], (step, rep["norms"])
    T = dp.tensors
    new = st.copy()
    new.x, new.F, new.be = T["x"].cpu().numpy(), T["F"].cpu().numpy(), T["be"].cpu().numpy()
    return du.cpu().numpy().reshape(-1, nd), new, rep


def _certificate(P, st, pat, bc, got, r0):
    fint, fext = O.forces(P, st, compact_to_full(P, pat, got))
    rr = (fint - fext)[pat.active]
    rr[O.constrained(P, st, pat, bc.mask)] = 0.0
    return np.linalg.norm(rr) / r0


def _trajectory(ctx, w, steps, tol, method, du_bound, label):
    st_o = w.particles
    st_g = w.particles.copy()
    P = w.prob
    worst, worst_c = 0.0, 0.0
    out = []
    for k in steps:
        bc = w.bc(k)
        dof, orep, pat = O.newton(P, st_o, bc.mask, bc.value, tol=tol)
        assert orep.converged, (label, k)
        got, st_g_new, rep = _gpu_step(ctx, w, st_g, k, tol, method)
        assert got.shape[0] == pat.n_row
        ref = dof[pat.active]
        if P.up:
            e = max(rel_err(got[:, :P.dim], ref[:, :P.dim]), rel_err(got[:, P.dim], ref[:, P.dim]))
        else:
            e = rel_err(got, ref)
        cert = _certificate(P, st_g, pat, bc, got, orep.norms[0][0]) if not P.up else 0.0
        print(f"  [{label}] step {k}: du rel err {e:.2e}, oracle residual at GPU du {cert:.2e}, "
              f"newton {rep['iters']} (oracle {orep.iters}), krylov {rep['krylov'][:rep['iters']]}", flush=True)
        worst, worst_c = max(worst, e), max(worst_c, cert)
        assert e <= du_bound, (label, k, e)
        assert cert <= 1e-9, (label, k, cert)
        out.append((k, got, pat))
        st_o = O.update(P, st_o, dof)
        st_g = st_g_new
    print(f"  [{label}] worst step du rel err {worst:.2e}, worst certificate {worst_c:.2e}", flush=True)
    return out, st_g


def terzaghi(z, t, cv, H, nterm=400):
    T = cv * t / H ** 2
    s = np.zeros_like(z)
    for m in range(nterm):
        M = math.pi * (2 * m + 1) / 2
        s += 2 / M * np.sin(M * z / H) * math.exp(-M * M * T)
    return s


def test_consolidation_100_steps_and_terzaghi(ctx):
    """u-p consolidation (10 kPa surface load, top drainage, dt = 1 s) on a
    64-cell-high column 8 cells wide: every step's displacement and pressure
    increments agree with the oracle, and the GPU's pore pressure along the
    centre line follows Terzaghi's solution (c_v = 0.013462 m^2/s, H = 1 m)."""
    w = W.make_c4(n=64, n_steps=100, width_cells=8)
    P = w.prob
    print(f"[traj] consolidation 8x64, {w.particles.np} particles", flush=True)
    out, _ = _trajectory(ctx, w, range(1, 101), 1e-12, 0, 1e-9, "u-p")
    E, nu = P.E, P.nu
    cv = P.perm / P.mu_f * E * (1 - nu) / ((1 + nu) * (1 - 2 * nu))
    assert abs(cv - 0.013462) < 1e-6
    idx = P.node_grid_index()
    for t in (10, 20, 50, 100):
        k, got, pat = out[t - 1]
        full = compact_to_full(P, pat, got)
        col = (idx[0] == P.n[0] // 2) & (idx[1] >= 1) & (idx[1] <= P.n[1] - 1)
        y = idx[1][col] * P.h
        p = full[col, 2]
        ref = 1e4 * terzaghi(1.0 - y, float(t), cv, 1.0)
        err = np.abs(p - ref).max() / 1e4
        print(f"  t = {t} s: max |p - Terzaghi| / p0 = {err:.3e}", flush=True)
        assert err < 2e-2, (t, err)


def _reading(w, push):
    w.prob.c = 1e3
    w.prob.dp_match = 4          # outer cone, associated flow
    w.footing = (w.footing[0], w.footing[1], w.footing[2], push)
    return w


def test_cube_footing_trajectory(ctx):
    """The 3-D footing on a 12^3 grid: geostatic step and five 0.1 mm
    pushes, solved on the GPU with the 3-D multigrid preconditioner."""
    w = _reading(W.make_c3(n=12, n_steps=5), -1e-4)
    print(f"[traj] cube 12^3, {w.particles.np} particles", flush=True)
    _trajectory(ctx, w, range(0, 6), 1e-12, 2, 1e-8, "cube")


def test_plane_strain_footing_full_size_trajectory(ctx):
    """The 256 x 128 plane-strain footing at full size: geostatic step and
    two 0.1 mm pushes with the multigrid preconditioner."""
    w = _reading(W.make_c2(n_steps=2), -1e-4)
    print(f"[traj] plane-strain footing 256x128, {w.particles.np} particles", flush=True)
    _trajectory(ctx, w, range(0, 3), 1e-12, 2, 1e-8, "footing")
