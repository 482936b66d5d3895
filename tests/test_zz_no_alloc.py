"""mpm_residual_noalloc (the residual whose force records live in the
library's fixed scratch array instead of context memory) against
mpm_residual on the same prepared problems: two calls in a row, the second
on a smaller problem, in plane strain and in 3-D.  Both run the same
kernels in the same order, so r, r_raw and the reactions must agree bit for
bit.  A problem whose records exceed the fixed array is rejected before
any launch."""
import numpy as np
import pytest

from paper_2507_09435_amd import workloads as W

from gpu_common import react_mask

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


def _both(ctx, w, step, seed):
    from paper_2507_09435_amd import mpm as M
    P, st = w.prob, w.particles
    dp = M.make_problem([(P, st)], [w.bc(step)], react_masks=[react_mask(w)])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n_row, nd)) * 2e-3 * P.h
    d[:, 1] -= 2e-3 * P.h
    du = torch.from_numpy(d.reshape(-1)).cuda()
    out = []
    for fn in (M.mpm_residual_noalloc, M.mpm_residual):
        r = torch.full((n_row * nd,), np.nan, dtype=torch.float64, device="cuda")
        rr = torch.full((n_row * nd,), np.nan, dtype=torch.float64, device="cuda")
        react = fn(ctx, dp, du, r, rr, want_reaction=True)
        torch.cuda.synchronize()
        out.append((r.cpu().numpy(), rr.cpu().numpy(), react))
    (a, ar, ae), (b, br, be) = out
    assert np.isfinite(a).all() and np.isfinite(ar).all()
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ar, br)
    np.testing.assert_array_equal(ae, be)
    return st.np


@pytest.mark.parametrize("dim", [2, 3])
def test_noalloc_residual_matches_twice(ctx, dim):
    """A larger problem, then a smaller one: the second call reuses the
    scratch the first one filled and must still match bit for bit."""
    print(f"[noalloc] dim={dim}", flush=True)
    if dim == 2:
        big, small = W.small_footing(n_y=24), W.small_footing(n_y=7)
    else:
        big, small = W.make_c3(n=16, n_steps=1), W.make_c3(n=8, n_steps=1)
    n1 = _both(ctx, big, 1, seed=71)
    n2 = _both(ctx, small, 1, seed=72)
    assert n2 < n1
    print(f"  {n1} then {n2} particles: bitwise equal to mpm_residual", flush=True)


def test_noalloc_residual_rejects_too_many_particles(ctx):
    """Records beyond the fixed array: INVALID from the host-side size
    check, and the context keeps working."""
    from paper_2507_09435_amd import mpm as M
    print("[noalloc] oversized problem", flush=True)
    w = W.small_footing(n_y=170)   # 8 * 170^2 = 231,200 particles x 160 B > 32 MiB
    assert w.particles.np * 160 > M.MPM_NOALLOC_SCRATCH_BYTES
    dp = M.make_problem([(w.prob, w.particles)], [w.bc(1)], react_masks=[react_mask(w)])
    n_row, nnzb, nd = M.mpm_prepare(ctx, dp)
    du = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    r = torch.zeros(n_row * nd, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MPMError) as ei:
        M.mpm_residual_noalloc(ctx, dp, du, r)
    assert ei.value.code == M.MPM_E_INVALID
    assert "scratch" in str(ei.value)
    _both(ctx, W.small_footing(n_y=6), 1, seed=73)
