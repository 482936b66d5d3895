"""Parity at the benchmark's full size and launch configuration: the
256x128-cell Drucker-Prager configuration (131072 particles).  The oracle
evaluates the whole residual and every Jacobian block, and runs the same
geostatic Newton step."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_09435_amd import workloads as W

from gpu_common import row_errors, block_errors, compact_to_full, react_mask, rel_err, seeded_du

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def c2():
    from paper_2507_09435_amd import mpm as M
    M.load()
    assert torch.cuda.is_available()
    w = W.make_c2(n_steps=1)
    ctx = M.mpm_create(0)
    dp = M.make_problem([(w.prob, w.particles)], [w.bc(0)], react_masks=[react_mask(w)])
    shape = M.mpm_prepare(ctx, dp)
    pat = O.pattern(w.prob, w.particles)
    yield w, ctx, dp, shape, pat
    M.mpm_destroy(ctx)


def test_full_pattern(c2):
    from paper_2507_09435_amd import mpm as M
    w, ctx, dp, (n_row, nnzb, nd), pat = c2
    print(f"[fullsize] pattern rows={n_row} blocks={nnzb}", flush=True)
    assert (n_row, nnzb) == (pat.n_row, pat.nnzb) == (33929, 836561)
    rowptr = torch.zeros(n_row + 1, dtype=torch.int32, device="cuda")
    colind = torch.zeros(nnzb, dtype=torch.int32, device="cuda")
    active = torch.zeros(n_row, dtype=torch.int64, device="cuda")
    M.mpm_jacobian_bsr(ctx, dp, None, rowptr, colind, None, active)
    torch.cuda.synchronize()
    assert np.array_equal(rowptr.cpu().numpy(), pat.rowptr)
    assert np.array_equal(colind.cpu().numpy(), pat.colind)
    assert np.array_equal(active.cpu().numpy(), pat.active)


def test_full_residual_and_jacobian(c2):
    from paper_2507_09435_amd import mpm as M
    w, ctx, dp, (n_row, nnzb, nd), pat = c2
    P, st = w.prob, w.particles
    print("[fullsize] residual + jacobian", flush=True)
    du = seeded_du(P, pat, seed=31, amp=1e-3)
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
    re = row_errors(rr.cpu().numpy(), ref, fint[pat.active], fext[pat.active])
    print(f"  worst row {re.max():.2e}", flush=True)
    assert re.max() <= 1e-10, (re.max(), int(re.argmax()))
    errs = block_errors(val.cpu().numpy(), O.jacobian_bsr(P, st, full, pat))
    assert errs.max() <= 1e-9, errs.max()


@pytest.mark.parametrize("method", [0, 2])
def test_full_geostatic_newton(c2, method):
    from paper_2507_09435_amd import mpm as M
    w, ctx, dp, (n_row, nnzb, nd), pat = c2
    P, st = w.prob, w.particles
    print(f"[fullsize] geostatic newton, krylov_method={method}", flush=True)
    du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    rep = M.mpm_newton_step(ctx, dp, du, tol=1e-12, commit=False, krylov_rtol=1e-12, krylov_method=method)
    print(f"  newton {rep['iters']} krylov {rep['krylov']} ms {rep['ms_total']:.1f}", flush=True)
    torch.cuda.synchronize()
    assert rep["converged"]
    bc = w.bc(0)
    dof, orep, _ = O.newton(P, st, bc.mask, bc.value, tol=1e-12, pat=pat)
    assert orep.converged
    got = du.cpu().numpy().reshape(-1, nd)
    e = rel_err(got, dof[pat.active])
    print(f"  du rel err {e:.3e}", flush=True)
    assert e <= 1e-10
