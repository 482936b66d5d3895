"""Parity at full size for the 3-D footing cube (128^3 cells, 8388608
particles, friction angle per particle).

* Pattern, all rows, bit-exact: two nodes a and a + d couple exactly when an
  occupied stencil origin o has both in o + {0,1,2}^3, i.e. when some origin
  lies in the per-axis window [a + max(d,0) - 2, a + min(d,0)].  Counting
  that over the origin occupancy grid gives every row's column list in
  ascending node order without forming particle pairs.
* Residual and Jacobian on sampled node boxes: a node's row only sees the
  particles whose origin lies within two cells below it, so the oracle
  evaluates that particle subset and the rows are complete.
* The geostatic Newton step converges, and the oracle's residual at the GPU
  solution vanishes on the sampled boxes."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_09435_amd import workloads as W

from gpu_common import block_errors, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# node-index boxes (inclusive, per axis x, y, z)
BOXES = [((60, 64), (60, 64), (60, 65)),     # under the footing, top of the layer
         ((-1, 2), (-1, 2), (-1, 2)),        # the base corner with its ghost nodes
         ((100, 103), (20, 23), (30, 33))]   # interior


def _window_any(occ, axis, lo, hi):
    """out[a] = any(occ[a + lo .. a + hi]) along one axis (outside: False)."""
    out = np.zeros_like(occ)
    n = occ.shape[axis]
    for s in range(lo, hi + 1):
        src = [slice(None)] * occ.ndim
        dst = [slice(None)] * occ.ndim
        if s >= 0:
            src[axis], dst[axis] = slice(s, n), slice(0, n - s)
        else:
            src[axis], dst[axis] = slice(0, n + s), slice(-s, n)
        out[tuple(dst)] |= occ[tuple(src)]
    return out


def counted_pattern(P, o):
    """Rows (active full-grid node ids), rowptr and colind (row indices) of
    the coupling pattern, from the origins o [3][np] alone."""
    npa = P.nodes_per_axis                                  # x, y, z
    occ = np.zeros(npa[::-1], dtype=bool)                   # indexed [z][y][x]
    occ[o[2] + 1, o[1] + 1, o[0] + 1] = True
    strides = np.array([1, npa[0], npa[0] * npa[1]], dtype=np.int64)
    offs = [(dx, dy, dz) for dz in range(-2, 3) for dy in range(-2, 3) for dx in range(-2, 3)]
    offs.sort(key=lambda d: d[0] * strides[0] + d[1] * strides[1] + d[2] * strides[2])

    def coupled(d):
        m = occ
        for ax, dd in zip((2, 1, 0), d):                    # array axis of x is 2
            m = _window_any(m, ax, max(dd, 0) - 2, min(dd, 0))
        return m.reshape(-1)

    act_mask = coupled((0, 0, 0))
    active = np.nonzero(act_mask)[0].astype(np.int64)
    row_of = np.full(act_mask.shape[0], -1, dtype=np.int64)
    row_of[active] = np.arange(active.shape[0])
    masks = [coupled(d)[active] for d in offs]
    cnt = np.zeros(active.shape[0], dtype=np.int64)
    for m in masks:
        cnt += m
    rowptr = np.concatenate([[0], np.cumsum(cnt)])
    colind = np.empty(rowptr[-1], dtype=np.int64)
    fill = rowptr[:-1].copy()
    for d, m in zip(offs, masks):
        lin = d[0] * strides[0] + d[1] * strides[1] + d[2] * strides[2]
        r = np.nonzero(m)[0]
        colind[fill[r]] = row_of[active[r] + lin]
        fill[r] += 1
    return active, rowptr, colind


def _subset(P, st, o, box):
    keep = np.ones(st.np, dtype=bool)
    for k, (lo, hi) in enumerate(box):
        keep &= (o[k] >= lo - 2) & (o[k] <= hi)
    cp = lambda a: None if a is None else a[..., keep].copy()
    return W.Particles(cp(st.x), cp(st.vol0), cp(st.F), cp(st.be), cp(st.fp), cp(st.E), cp(st.phi))


def _box_nodes(P, box):
    idx = P.node_grid_index()
    sel = np.ones(P.n_nodes, dtype=bool)
    for k, (lo, hi) in enumerate(box):
        sel &= (idx[k] >= lo) & (idx[k] <= hi)
    return np.nonzero(sel)[0]


@pytest.fixture(scope="module")
def c3():
    from paper_2507_09435_amd import mpm as M
    M.load()
    assert torch.cuda.is_available()
    print("[c3] building the 128^3 workload", flush=True)
    w = W.make_c3()
    ctx = M.mpm_create(0)
    dp = M.make_problem([(w.prob, w.particles)], [w.bc(0)])
    shape = M.mpm_prepare(ctx, dp)
    o = O.origins(w.prob, w.particles)
    n_row, nnzb, nd = shape
    rowptr = torch.zeros(n_row + 1, dtype=torch.int32, device="cuda")
    colind = torch.zeros(nnzb, dtype=torch.int32, device="cuda")
    active = torch.zeros(n_row, dtype=torch.int64, device="cuda")
    M.mpm_jacobian_bsr(ctx, dp, None, rowptr, colind, None, active)
    torch.cuda.synchronize()
    pat = (active.cpu().numpy(), rowptr.cpu().numpy(), colind.cpu().numpy())
    yield w, ctx, dp, shape, o, pat
    M.mpm_destroy(ctx)


def test_c3_pattern_counted(c3):
    w, ctx, dp, (n_row, nnzb, nd), o, (act, rp, ci) = c3
    print(f"[c3] pattern rows={n_row} blocks={nnzb}", flush=True)
    # closed form for a box of occupied origins: nodes -1..129 in x and y,
    # -1..65 in z; per axis n nodes give 5n - 6 pairs within distance 2
    assert (n_row, nnzb) == (131 * 131 * 67, (5 * 131 - 6) ** 2 * (5 * 67 - 6))
    active, rowptr, colind = counted_pattern(w.prob, o)
    assert (n_row, nnzb) == (active.shape[0], colind.shape[0])
    assert np.array_equal(act, active)
    assert np.array_equal(rp, rowptr)
    assert np.array_equal(ci, colind)


def _sampled_rows(P, st, o, act, du_full):
    """Per box: (box, its active nodes, their GPU rows, the particle subset,
    oracle residual rows, oracle f_int rows)."""
    row_of = np.full(P.n_nodes, -1, dtype=np.int64)
    row_of[act] = np.arange(act.shape[0])
    for box in BOXES:
        sub = _subset(P, st, o, box)
        nodes = _box_nodes(P, box)
        nodes = nodes[row_of[nodes] >= 0]
        fint, fext = O.forces(P, sub, du_full)
        yield box, nodes, row_of[nodes], sub, (fint - fext)[nodes], fint[nodes]


def test_c3_sampled_residual_and_jacobian(c3):
    from paper_2507_09435_amd import mpm as M
    w, ctx, dp, (n_row, nnzb, nd), o, (act, rp, ci) = c3
    P, st = w.prob, w.particles
    rng = np.random.default_rng(41)
    du_full = rng.normal(size=(P.n_nodes, 3)) * 1e-3 * P.h
    du = torch.from_numpy(np.ascontiguousarray(du_full[act]).reshape(-1)).cuda()
    rr = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    M.mpm_residual(ctx, dp, du, None, rr)
    val = torch.zeros(nnzb * 9, dtype=torch.float64, device="cuda")
    M.mpm_jacobian_bsr(ctx, dp, du, val=val, raw=True)
    torch.cuda.synchronize()
    rgpu = rr.cpu().numpy().reshape(-1, 3)
    for box, nodes, rows, sub, ref, fint in _sampled_rows(P, st, o, act, du_full):
        print(f"[c3] box {box}: {nodes.shape[0]} rows, {sub.np} particles", flush=True)
        e = rel_err(rgpu[rows], ref, max(np.linalg.norm(ref), np.linalg.norm(fint)))
        assert e <= 1e-10, e
        spat = O.pattern(P, sub)
        jref = O.jacobian_bsr(P, sub, du_full, spat)
        for node, r in zip(nodes, rows):
            rs = spat.row_of_node[node]
            cols_ref = spat.active[spat.colind[spat.rowptr[rs]:spat.rowptr[rs + 1]]]
            assert np.array_equal(cols_ref, act[ci[rp[r]:rp[r + 1]]])
            vg = val[int(rp[r]) * 9:int(rp[r + 1]) * 9].cpu().numpy().reshape(-1, 3, 3)
            assert block_errors(vg, jref[spat.rowptr[rs]:spat.rowptr[rs + 1]]).max() <= 1e-9


def test_c3_geostatic_newton(c3):
    from paper_2507_09435_amd import mpm as M
    w, ctx, dp, (n_row, nnzb, nd), o, (act, rp, ci) = c3
    P, st = w.prob, w.particles
    print("[c3] geostatic newton", flush=True)
    du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    rep = M.mpm_newton_step(ctx, dp, du, tol=1e-10, commit=False, krylov_rtol=1e-12)
    torch.cuda.synchronize()
    print(f"  newton {rep['iters']} krylov {rep['krylov']} ms {rep['ms_total']:.1f}", flush=True)
    assert rep["converged"], rep
    got = du.cpu().numpy().reshape(-1, nd)
    du_full = np.zeros((P.n_nodes, 3))
    du_full[act] = got
    bc = w.bc(0)
    r0 = rep["norms"][0]
    for box, nodes, rows, sub, ref, fint in _sampled_rows(P, st, o, act, du_full):
        ref = ref.copy()
        ref[bc.mask[nodes].astype(bool)] = 0.0
        print(f"  box {box}: oracle |r| {np.linalg.norm(ref):.3e} (r0 {r0:.3e})", flush=True)
        assert np.linalg.norm(ref) <= 1e-9 * r0
