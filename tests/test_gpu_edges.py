"""Edge cases of the HIP path through the C ABI: degenerate inputs the method
admits (one particle, an empty sim inside a batch, a problem without
particles, particles on the lines where the stencil origin changes, the
outermost origins the padded grid allows) against the oracle, and the
inputs the library must reject (non-finite or out-of-grid coordinates,
options out of range) with their status codes and an intact context."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_09435_amd import workloads as W

from gpu_common import (row_errors, block_errors, compact_to_full, oracle_pattern_batch, react_mask, rel_err, seeded_du)

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


def _with_particles(w, x):
    """The workload w with its particles replaced by undeformed ones at x."""
    P = w.prob
    st = W.identity_state(P.dim, np.ascontiguousarray(x, dtype=np.float64), P.h, 4 if P.dim == 2 else 8)
    return W.Workload(P, st, w.n_steps, w.geostatic, w.walls, w.footing, w.p_drained)


def _pattern(ctx, dp, n_row, nnzb):
    from paper_2507_09435_amd import mpm as M
    rowptr = torch.zeros(n_row + 1, dtype=torch.int32, device="cuda")
    colind = torch.zeros(max(nnzb, 1), dtype=torch.int32, device="cuda")
    active = torch.zeros(max(n_row, 1), dtype=torch.int64, device="cuda")
    M.mpm_jacobian_bsr(ctx, dp, None, rowptr, colind, None, active)
    torch.cuda.synchronize()
    return active.cpu().numpy()[:n_row], rowptr.cpu().numpy(), colind.cpu().numpy()[:nnzb]


def _check_parity(ctx, w, step, seed):
    """Pattern bit-exact, residual within 1e-10 and raw Jacobian blocks
    within 1e-9 of the oracle at a seeded increment."""
    from paper_2507_09435_amd import mpm as M
    P, st = w.prob, w.particles
    dp = M.make_problem([(P, st)], [w.bc(step)], react_masks=[react_mask(w)])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    pat = O.pattern(P, st)
    assert (n_row, nnzb, nd) == (pat.n_row, pat.nnzb, P.ndof)
    act, rp, ci = _pattern(ctx, dp, n_row, nnzb)
    np.testing.assert_array_equal(act, pat.active)
    np.testing.assert_array_equal(rp, pat.rowptr)
    np.testing.assert_array_equal(ci, pat.colind)
    du = seeded_du(P, pat, seed=seed)
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
    assert rel_err(rr.cpu().numpy().reshape(-1, nd), ref, scale) <= 1e-10
    assert row_errors(rr.cpu().numpy(), ref, fint[pat.active], fext[pat.active]).max() <= 1e-10
    jref = O.jacobian_bsr(P, st, full, pat)
    assert block_errors(val.cpu().numpy(), jref).max() <= 1e-9


# ----------------------------------------------------------- one particle --
@pytest.mark.parametrize("name", ["plane", "plane_cell_centre", "up", "cube"])
def test_single_particle(ctx, name):
    """One particle: a single stencil group, 3^d rows, each coupled to all
    3^d nodes of the stencil (2-D records path, u-p path, 3-D path)."""
    print(f"[edge] single particle case={name}", flush=True)
    if name.startswith("plane"):
        w = W.small_footing(n_y=6)
        # a cell centre is where floor(u - 1/2) steps: the outer weight is 0
        x = [[0.37], [0.21]] if name == "plane" else [[5.5 * w.prob.h], [2.5 * w.prob.h]]
        step = 1
    elif name == "up":
        w = W.make_c4(n=8, n_steps=1, width_cells=4, dt=1.0)
        x = [[0.31], [0.52]]
        step = 1
    else:
        w = W.make_c3(n=8, n_steps=1)
        x = [[0.41], [0.56], [0.23]]
        step = 1
    w = _with_particles(w, np.array(x))
    _check_parity(ctx, w, step, seed=31)


# --------------------------------------------- stencil-origin boundaries ---
def test_particles_on_origin_switch_lines(ctx):
    """Particles on every node line and every cell-centre line of a footing
    grid with h = 1/12 (not a power of two, so (x - x0)/h rounds), plus the
    outermost positions whose origins are still inside the padded grid
    (origin -1 at x0 - h/2 and origin n-1 just below x0 + (n + 1/2) h)."""
    print("[edge] particles on origin switch lines", flush=True)
    w = W.small_footing(n_y=6)
    P = w.prob
    h = P.h
    axes = []
    for k in range(2):
        n = P.n[k]
        vals = [P.x0[k] + 0.5 * i * h for i in range(0, 2 * n + 1)]
        vals += [P.x0[k] - 0.5 * h, np.nextafter(P.x0[k] + (n + 0.5) * h, -np.inf)]
        axes.append(np.array(vals))
    gx, gy = np.meshgrid(axes[0], axes[1], indexing="xy")
    x = np.stack([gx.reshape(-1), gy.reshape(-1)])
    w = _with_particles(w, x)
    o = O.origins(P, w.particles)
    for k in range(2):   # the set reaches both ends of the allowed origin range
        assert o[k].min() == -1 and o[k].max() == P.n[k] - 1
    _check_parity(ctx, w, 1, seed=32)


# ------------------------------------------------------------ empty sims ---
def _empty_like(w):
    """w without particles (per-particle loads kept as empty arrays, so that
    a batch keeps the other sims' loads)."""
    P = w.prob
    st = W.Particles(np.zeros((P.dim, 0)), np.zeros(0), np.zeros((P.dim * P.dim, 0)),
                     np.zeros((4 if P.dim == 2 else 6, 0)))
    if w.particles.fp is not None:
        st.fp = np.zeros((w.particles.fp.shape[0], 0))
    return W.Workload(P, st, w.n_steps, w.geostatic, w.walls, w.footing, w.p_drained)


@pytest.mark.parametrize("method", [0, 2])
def test_empty_sims_in_batch(ctx, method):
    """Sims without particles at the front, middle and end of a batch: they
    own no rows, report zero reaction and converge at iteration 0, and the
    other sims match their own oracle (pattern, residual, Newton)."""
    from paper_2507_09435_amd import mpm as M
    print(f"[edge] empty sims in a batch, krylov_method={method}", flush=True)
    ws = []
    for k, (n_y, empty) in enumerate(((3, True), (4, False), (5, True), (5, False), (4, True))):
        w = W.small_footing(n_y=n_y)
        w.prob.dp = 0
        if empty:
            w = _empty_like(w)
        else:
            w.particles.E = np.full(w.particles.np, 10.0 ** (6.5 + 0.25 * k))
        ws.append(w)
    sims = [(w.prob, w.particles) for w in ws]
    dp = M.make_problem(sims, [w.bc(1) for w in ws], react_masks=[react_mask(w) for w in ws])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    act, rp, ci, pats = oracle_pattern_batch(sims)
    g_act, g_rp, g_ci = _pattern(ctx, dp, n_row, nnzb)
    np.testing.assert_array_equal(g_act, act)
    np.testing.assert_array_equal(g_rp, rp)
    np.testing.assert_array_equal(g_ci, ci)

    dus = [seeded_du(w.prob, pat, seed=40 + k) for k, (w, pat) in enumerate(zip(ws, pats))]
    du = torch.from_numpy(np.concatenate([d.reshape(-1) for d in dus])).cuda()
    rr = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    react = M.mpm_residual(ctx, dp, du, None, rr, want_reaction=True)
    torch.cuda.synchronize()
    got = rr.cpu().numpy().reshape(-1, nd)
    off = 0
    for k, (w, pat) in enumerate(zip(ws, pats)):
        if pat.n_row == 0:
            assert react[k] == 0.0
            continue
        fint, fext = O.forces(w.prob, w.particles, compact_to_full(w.prob, pat, dus[k]))
        ref = (fint - fext)[pat.active]
        assert rel_err(got[off:off + pat.n_row], ref, max(np.linalg.norm(ref), np.linalg.norm(fint[pat.active]))) \
            <= 1e-10
        off += pat.n_row

    du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    rep = M.mpm_newton_step(ctx, dp, du, tol=1e-13, max_iter=25, commit=False, krylov_rtol=1e-12,
                            krylov_method=method)
    torch.cuda.synchronize()
    assert rep["converged"] and all(rep["sim_converged"]), rep
    got = du.cpu().numpy().reshape(-1, nd)
    off = 0
    for k, (w, pat) in enumerate(zip(ws, pats)):
        if pat.n_row == 0:
            assert rep["sim_iters"][k] == 0 and rep["sim_reaction"][k] == 0.0
            continue
        bc = w.bc(1)
        dof, orep, _ = O.newton(w.prob, w.particles, bc.mask, bc.value, tol=1e-13)
        assert orep.converged
        e = rel_err(got[off:off + pat.n_row], dof[pat.active])
        print(f"  sim {k}: du rel err {e:.3e}", flush=True)
        assert e <= 1e-10
        off += pat.n_row


@pytest.mark.parametrize("kind", ["cube", "up"])
def test_empty_sims_under_3x3_multigrid(ctx, kind):
    """Sims without particles around two sims of different size under the
    3x3-block multigrid (3-D and u-p): the empty sims own no rows, get no
    levels and converge at iteration 0 (their dense coarsest block is
    empty), and each other sim's increment matches its own oracle Newton
    solution."""
    from paper_2507_09435_amd import mpm as M
    print(f"[edge] empty sims under the 3x3-block multigrid, kind={kind}", flush=True)
    if kind == "cube":
        full = [W.make_c3(n=n, n_steps=1) for n in (8, 10)]
        for w in full:
            w.particles.phi = np.full(w.particles.np, np.radians(40.0))   # the geostatic state stays elastic
        step = 0
    else:
        full = [W.make_c4(n=n, n_steps=1, width_cells=n, dt=1.0) for n in (12, 16)]
        step = 1
    ws = [_empty_like(full[0]), full[0], _empty_like(full[1]), full[1], _empty_like(full[0])]
    dp = M.make_problem([(w.prob, w.particles) for w in ws], [w.bc(step) for w in ws])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    rep = M.mpm_newton_step(ctx, dp, du, tol=1e-12, max_iter=25, commit=False, krylov_rtol=1e-12, krylov_method=2)
    torch.cuda.synchronize()
    assert rep["converged"] and all(rep["sim_converged"]), rep
    print(f"  newton {rep['iters']}  krylov {rep['krylov'][:rep['iters']]}", flush=True)
    got = du.cpu().numpy().reshape(-1, nd)
    off = 0
    for k, w in enumerate(ws):
        if w.particles.np == 0:
            assert rep["sim_iters"][k] == 0
            continue
        bc = w.bc(step)
        dof, orep, pat = O.newton(w.prob, w.particles, bc.mask, bc.value, tol=1e-12)
        assert orep.converged
        # bound widened only to 10x the oracle's own spread at its round-off floor
        more, _, _ = O.newton(w.prob, w.particles, bc.mask, bc.value, tol=1e-30, stall_factor=0.0,
                              maxit=orep.iters + 4, dof0_full=dof)
        g, r, m = got[off:off + pat.n_row], dof[pat.active], more[pat.active]
        if kind == "up":
            e = max(rel_err(g[:, :2], r[:, :2]), rel_err(g[:, 2], r[:, 2]))
            spread = max(rel_err(m[:, :2], r[:, :2]), rel_err(m[:, 2], r[:, 2]))
        else:
            e, spread = rel_err(g, r), rel_err(m, r)
        b = max(1e-10, 10.0 * spread)
        print(f"  sim {k}: du rel err {e:.3e} (bound {b:.1e})", flush=True)
        assert e <= b
        off += pat.n_row
    assert off == n_row


@pytest.mark.parametrize("method", [0, 2])
def test_problem_without_particles(ctx, method):
    """No particles at all: no rows, no blocks; the residual, pattern,
    Newton step (converged at iteration 0) and update accept the empty
    (NULL) vectors."""
    from paper_2507_09435_amd import mpm as M
    print(f"[edge] problem without particles, krylov_method={method}", flush=True)
    w = _empty_like(W.small_footing(n_y=4))
    dp = M.make_problem([(w.prob, w.particles)], [w.bc(1)])
    assert M.mpm_prepare(ctx, dp) == (0, 0, 2)
    react = M.mpm_residual(ctx, dp, None, None, want_reaction=True)
    assert react[0] == 0.0
    rowptr = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    M.mpm_jacobian_bsr(ctx, dp, None, rowptr=rowptr)
    torch.cuda.synchronize()
    assert int(rowptr.item()) == 0
    rep = M.mpm_newton_step(ctx, dp, None, commit=False, krylov_method=method)
    assert rep["converged"] and rep["iters"] == 0 and rep["krylov_iters"] == 0
    M.mpm_update(ctx, dp, None, None, None, None)
    # a committed step advances the problem's state: the context needs a new prepare
    rep = M.mpm_newton_step(ctx, dp, None, commit=True, krylov_method=method)
    assert rep["converged"]
    with pytest.raises(M.MPMError) as ei:
        M.mpm_update(ctx, dp, None, None, None, None)
    assert ei.value.code == M.MPM_E_INVALID


# ------------------------------------------------------- rejected inputs ---
@pytest.mark.parametrize("kind", ["nan", "inf", "below", "above"])
def test_prepare_rejects_bad_coordinates(ctx, kind):
    """A non-finite coordinate gives NONFINITE and an origin outside
    -1..n-1 gives OUT_OF_GRID; afterwards the context holds no prepared
    problem (INVALID) and prepares the next valid problem correctly."""
    from paper_2507_09435_amd import mpm as M
    print(f"[edge] bad coordinate kind={kind}", flush=True)
    w = W.small_footing(n_y=4)
    P = w.prob
    bad = w.particles.copy()
    axis, p = 1, 7
    bad.x[axis, p] = {"nan": np.nan, "inf": np.inf,
                      "below": P.x0[axis] - (0.5 + 2.0 ** -20) * P.h,
                      "above": P.x0[axis] + (P.n[axis] + 0.5) * P.h}[kind]
    want = M.MPM_E_NONFINITE if kind in ("nan", "inf") else M.MPM_E_OUT_OF_GRID
    dpb = M.make_problem([(P, bad)], [w.bc(1)])
    with pytest.raises(M.MPMError) as ei:
        M.mpm_prepare(ctx, dpb)
    assert ei.value.code == want
    du = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MPMError) as ei:
        M.mpm_residual(ctx, dpb, du, None)
    assert ei.value.code == M.MPM_E_INVALID
    _check_parity(ctx, w, 1, seed=33)


def test_invalid_options_and_arguments(ctx):
    """Options and arguments out of range give INVALID without launching
    anything; the context stays usable."""
    from paper_2507_09435_amd import mpm as M
    print("[edge] invalid options", flush=True)

    def code(fn, *a, **k):
        with pytest.raises(M.MPMError) as ei:
            fn(*a, **k)
        return ei.value.code

    w = W.small_footing(n_y=4)
    dp = M.make_problem([(w.prob, w.particles)], [w.bc(1)])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    assert code(M.mpm_newton_step, ctx, dp, du, krylov_method=5) == M.MPM_E_INVALID
    assert code(M.mpm_newton_step, ctx, dp, du, krylov_method=-1) == M.MPM_E_INVALID
    assert code(M.mpm_newton_step, ctx, dp, du, tol=0.0) == M.MPM_E_INVALID
    assert code(M.mpm_newton_step, ctx, dp, du, max_iter=-1) == M.MPM_E_INVALID
    assert code(M.mpm_residual, ctx, dp, None, None) == M.MPM_E_INVALID          # rows exist: du required
    val = torch.zeros(nnzb * 4, dtype=torch.float64, device="cuda")
    x = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    assert code(M.mpm_spmv, ctx, val, x, x) == M.MPM_E_INVALID                  # y aliases x
    # a problem other than the prepared one
    w2 = W.small_footing(n_y=5)
    dp2 = M.make_problem([(w2.prob, w2.particles)], [w2.bc(1)])
    assert code(M.mpm_residual, ctx, dp2, du, None) == M.MPM_E_INVALID
    # material constants out of range are rejected by prepare
    for field, v in (("nu", 0.5), ("dp_match", 3), ("E", 0.0)):
        wb = W.small_footing(n_y=4)
        setattr(wb.prob, field, v)
        dpb = M.make_problem([(wb.prob, wb.particles)], [wb.bc(1)])
        assert code(M.mpm_prepare, ctx, dpb) == M.MPM_E_INVALID, field
    # sim ranges that do not tile the particles
    ws = [W.small_footing(n_y=4), W.small_footing(n_y=4)]
    dpb = M.make_problem([(v.prob, v.particles) for v in ws], [v.bc(1) for v in ws])
    n0 = ws[0].particles.np
    dpb.sim_start[1] = 2 * n0 + 1                       # beyond the next start
    assert code(M.mpm_prepare, ctx, dpb) == M.MPM_E_INVALID
    dpb.sim_start[1] = n0
    dpb.sim_start[2] = 2 * n0 - 1                       # does not end at np
    assert code(M.mpm_prepare, ctx, dpb) == M.MPM_E_INVALID
    # the Neo-Hookean law is elastic; J2 needs a yield strength
    for change in ({"elastic": 1, "dp": 1}, {"dp": 1, "dp_match": 3, "c": 0.0}, {"elastic": 2}, {"shape": 2},
                   {"shape": 1, "lp0": (0.0, 0.0, 0.0)}):
        wb = W.small_footing(n_y=4)
        for k, v in change.items():
            setattr(wb.prob, k, v)
        dpb = M.make_problem([(wb.prob, wb.particles)], [wb.bc(1)])
        assert code(M.mpm_prepare, ctx, dpb) == M.MPM_E_INVALID, change
    # a device that does not exist
    with pytest.raises(M.MPMError):
        M.mpm_create(torch.cuda.device_count() + 3, stream=0)
    # the context still works
    _check_parity(ctx, w, 1, seed=34)
