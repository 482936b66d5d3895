"""Matrix-free Jacobian-vector products (the matrix-free Newton-Krylov
variant of Sec. 2.2, Remark 2) against the assembled BSR SpMV of the same
step, raw and Dirichlet-modified, in plane strain and in 3-D, and against
the oracle's Jacobian applied to the same vector."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_09435_amd import workloads as W

from gpu_common import compact_to_full, react_mask, rel_err, seeded_du

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
        return W.small_footing(n_y=8), 1
    if name == "c3small":
        return W.make_c3(n=8, n_steps=1), 0
    if name == "c3mid":
        return W.make_c3(n=16, n_steps=1), 0
    raise KeyError(name)


@pytest.mark.parametrize("name", ["footing", "c3small", "c3mid"])
@pytest.mark.parametrize("raw", [True, False])
def test_jv_matches_bsr_spmv(ctx, name, raw):
    from paper_2507_09435_amd import mpm as M
    print(f"[jv] case={name} raw={raw}", flush=True)
    w, step = _case(name)
    P, st = w.prob, w.particles
    dp = M.make_problem([(P, st)], [w.bc(step)], react_masks=[react_mask(w)])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    pat = O.pattern(P, st)
    du = seeded_du(P, pat, seed=51)
    dut = torch.from_numpy(du.reshape(-1)).cuda()
    val = torch.zeros(nnzb * nd * nd, dtype=torch.float64, device="cuda")
    M.mpm_jacobian_bsr(ctx, dp, dut, val=val, raw=raw)
    x = torch.from_numpy(np.random.default_rng(52).normal(size=n_row * nd)).cuda()
    y_ref = torch.zeros_like(x)
    M.mpm_spmv(ctx, val, x, y_ref)
    y_new = torch.full_like(x, np.nan)
    M.mpm_jv(ctx, dp, dut, x, y_new, raw=raw)              # tangent tables recomputed at du
    y_reuse = torch.full_like(x, np.nan)
    M.mpm_jv(ctx, dp, None, x, y_reuse, raw=raw, reuse=True)
    torch.cuda.synchronize()
    a, b, c = y_ref.cpu().numpy(), y_new.cpu().numpy(), y_reuse.cpu().numpy()
    e = rel_err(b, a)
    print(f"  ||Jv - BSR x|| / ||BSR x|| = {e:.2e}", flush=True)
    assert e <= 1e-12
    np.testing.assert_array_equal(b, c)
    if raw and name != "c3mid":
        # the oracle's raw Jacobian applied to the same x
        jo = O.bsr_to_scipy(pat, O.jacobian_bsr(P, st, compact_to_full(P, pat, du), pat), nd) @ x.cpu().numpy()
        assert rel_err(b, jo) <= 1e-10


def test_jv_rejects_stale_or_up(ctx):
    from paper_2507_09435_amd import mpm as M
    w = W.make_c4(n=8, n_steps=1, width_cells=4, dt=1.0)
    dp = M.make_problem([(w.prob, w.particles)], [w.bc(1)])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    x = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(M.MPMError) as ei:
        M.mpm_jv(ctx, dp, x, x.clone(), y)
    assert ei.value.code == M.MPM_E_INVALID
    w2, step = _case("footing")
    dp2 = M.make_problem([(w2.prob, w2.particles)], [w2.bc(step)])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp2)
    x = torch.ones(n_row * nd, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(M.MPMError) as ei:
        M.mpm_jv(ctx, dp2, None, x, y, reuse=True)   # nothing assembled since this prepare
    assert ei.value.code == M.MPM_E_INVALID
