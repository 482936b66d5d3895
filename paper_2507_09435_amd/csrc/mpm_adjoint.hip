// Adjoint of one converged load step (plane strain, single-phase).
//
// Forward step: r_f(du; s, theta) = 0 on the free unknowns (Sec. 2.2), the
// reaction R = -sum over the reaction unknowns of the raw residual, and the
// particle update s' = S(du; s, theta).  Given dL/dR (per sim) and dL/ds'
// (per particle), the step's adjoint is
//   g      = mu^T dr/d(du) + sbar'^T dS/d(du)        (mu = -dL/dR on reaction rows)
//   J^T lambda = g          on the free unknowns      (one transposed solve)
//   sbar   = nu^T dr/ds     + sbar'^T dS/ds           (nu = mu - lambda)
//   thetab = nu^T dr/dtheta + sbar'^T dS/dtheta
// This replaces the paper's reverse pass through a tape of the whole run
// (Sec. 4.5) by one transposed solve per converged step.  The per-particle
// products are formed by forward-mode directional passes of the same
// particle function (one direction per particle input), so they are exact.
#include "mpm_internal.hpp"

namespace mpm {

struct AdjArgs {
  int64_t np;
  int nd;
  int dp, match;
  const double *xs, *vs, *Fs, *bes, *Es, *phis;
  const int32_t* psim;
  const int32_t* perm;
  const SimDev* sims;
  const int32_t* node_map;
  const double* fp_user;   // caller order
  double E, nu, phi, c, psi, apex_reg, rho0, g[3];
};

// Directional derivative, along input `dir`, of
//   sum_a nu_a . r_a(du, s, theta) + sbar' . S(du, s, theta)
// for one particle.  dir: 0..17 = du of local node a = dir/2, component dir%2;
// 18,19 = x; 20..23 = F (row-major); 24..27 = b^e (xx, yy, xy, zz); 28 = E; 29 = phi.
__device__ double adj_dir2(const AdjArgs& A, int64_t i, const double* __restrict__ du,
                           const double* __restrict__ nu_c, const double sbar[10], int dir) {
  const int64_t np = A.np;
  const SimDev& S = A.sims[A.psim[i]];
  dnum x[2];
  for (int k = 0; k < 2; ++k) x[k] = dnum(A.xs[k * np + i], dir == 18 + k ? 1.0 : 0.0);
  dnum Fn[2][2];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) Fn[r][c] = dnum(A.Fs[(r * 2 + c) * np + i], dir == 20 + r * 2 + c ? 1.0 : 0.0);
  Sym2<dnum> be{dnum(A.bes[0 * np + i], dir == 24 ? 1.0 : 0.0), dnum(A.bes[1 * np + i], dir == 25 ? 1.0 : 0.0),
                dnum(A.bes[2 * np + i], dir == 26 ? 1.0 : 0.0), dnum(A.bes[3 * np + i], dir == 27 ? 1.0 : 0.0)};
  dnum E(A.Es ? A.Es[i] : A.E, dir == 28 ? 1.0 : 0.0);
  dnum phi(A.phis ? A.phis[i] : A.phi, dir == 29 ? 1.0 : 0.0);
  // stencil: origin from the value (as in the forward kernels), weights as functions of x
  int32_t o[2];
  dnum w[2][3], dw[2][3];
  for (int k = 0; k < 2; ++k) {
    dnum u = (x[k] - S.x0[k]) / S.h;
    double of = floor(u.v - 0.5);
    o[k] = (int32_t)of;
    bspline3<dnum>(u - of, S.inv_h, w[k], dw[k]);
  }
  int32_t row[9];
  dnum dF[2][2] = {{dnum(1.0), dnum(0.0)}, {dnum(0.0), dnum(1.0)}};
  dnum xn[2] = {x[0], x[1]};
  for (int a = 0; a < 9; ++a) {
    const int ax = a % 3, ay = a / 3;
    int64_t node = S.node_base + (o[0] + ax + 1) + (int64_t)S.nna[0] * (o[1] + ay + 1);
    row[a] = A.node_map[node];
    dnum wa = w[0][ax] * w[1][ay];
    dnum g0 = dw[0][ax] * w[1][ay], g1 = w[0][ax] * dw[1][ay];
    for (int q = 0; q < 2; ++q) {
      dnum uq(du[(int64_t)row[a] * A.nd + q], dir == a * 2 + q ? 1.0 : 0.0);
      dF[q][0] += uq * g0;
      dF[q][1] += uq * g1;
      xn[q] += wa * uq;
    }
  }
  Mat<dnum> m = make_mat<dnum>(E, A.nu, phi, A.c, A.psi, A.dp, A.match, A.apex_reg);
  UpPar u0{0.0, 0.0, 0.0, 0.0, {0.0, 0.0, 0.0}};
  Out2<dnum> out;
  Sym2<dnum> b;
  dnum zero(0.0), gp0[2] = {dnum(0.0), dnum(0.0)};
  mech2<dnum>(m, dF, be, dnum(1.0), 0, u0, zero, gp0, out, &b);
  const double v0 = A.vs[i];
  const int64_t p = A.perm[i];
  double fpx = 0.0, fpy = 0.0;
  if (A.fp_user) { fpx = A.fp_user[0 * np + p]; fpy = A.fp_user[1 * np + p]; }
  const double mgx = A.rho0 * v0 * A.g[0] + fpx, mgy = A.rho0 * v0 * A.g[1] + fpy;
  double acc = 0.0;
  for (int a = 0; a < 9; ++a) {
    const int ax = a % 3, ay = a / 3;
    const double* nv = nu_c + (int64_t)row[a] * A.nd;
    if (nv[0] == 0.0 && nv[1] == 0.0) continue;
    dnum wa = w[0][ax] * w[1][ay];
    dnum g0 = dw[0][ax] * w[1][ay], g1 = w[0][ax] * dw[1][ay];
    dnum r0 = v0 * (out.P[0][0] * g0 + out.P[0][1] * g1) - wa * mgx;
    dnum r1 = v0 * (out.P[1][0] * g0 + out.P[1][1] * g1) - wa * mgy;
    acc += nv[0] * r0.d + nv[1] * r1.d;
  }
  bool any_s = false;
  for (int k = 0; k < 10; ++k) any_s = any_s || sbar[k] != 0.0;
  if (any_s) {
    acc += sbar[0] * xn[0].d + sbar[1] * xn[1].d;
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) {
        dnum f = dF[r][0] * Fn[0][c] + dF[r][1] * Fn[1][c];
        acc += sbar[2 + r * 2 + c] * f.d;
      }
    acc += sbar[6] * b.xx.d + sbar[7] * b.yy.d + sbar[8] * b.xy.d + sbar[9] * b.zz.d;
  }
  return acc;
}

__device__ __forceinline__ void load_sbar(const double* __restrict__ sbar_next, int64_t np, int64_t p, double sb[10]) {
  for (int k = 0; k < 10; ++k) sb[k] = sbar_next ? sbar_next[k * np + p] : 0.0;
}

// Pass 1: g += mu^T dr/d(du) + sbar'^T dS/d(du) per particle (18 directions).
__global__ void __launch_bounds__(128) k_adj_g2(AdjArgs A, const double* __restrict__ du,
                                               const double* __restrict__ mu, const double* __restrict__ sbar_next,
                                               double* __restrict__ g) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.np) return;
  double sb[10];
  load_sbar(sbar_next, A.np, A.perm[i], sb);
  const SimDev& S = A.sims[A.psim[i]];
  int32_t o[2];
  for (int k = 0; k < 2; ++k) o[k] = (int32_t)floor((A.xs[k * A.np + i] - S.x0[k]) / S.h - 0.5);
  for (int dir = 0; dir < 18; ++dir) {
    double v = adj_dir2(A, i, du, mu, sb, dir);
    if (v == 0.0) continue;
    const int a = dir / 2, q = dir % 2;
    int64_t node = S.node_base + (o[0] + a % 3 + 1) + (int64_t)S.nna[0] * (o[1] + a / 3 + 1);
    atomicAdd(&g[(int64_t)A.node_map[node] * A.nd + q], v);
  }
}

// Pass 2: state and parameter adjoints (12 directions); sbar_n in caller
// order, theta per particle in sorted order.
__global__ void __launch_bounds__(128) k_adj_s2(AdjArgs A, const double* __restrict__ du,
                                               const double* __restrict__ nu_c, const double* __restrict__ sbar_next,
                                               double* __restrict__ sbar_n, double* __restrict__ theta_p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.np) return;
  const int64_t p = A.perm[i];
  double sb[10];
  load_sbar(sbar_next, A.np, p, sb);
  for (int k = 0; k < 12; ++k) {
    double v = adj_dir2(A, i, du, nu_c, sb, 18 + k);
    if (k < 10) {
      if (sbar_n) sbar_n[k * A.np + p] = v;
    } else {
      theta_p[(int64_t)(k - 10) * A.np + i] = v;
    }
  }
}

// mu = -dL/dR on the reaction unknowns of each sim.
__global__ void k_adj_mu(const RowBlock* __restrict__ blocks, int nd, const uint8_t* __restrict__ rmask,
                         const double* __restrict__ rbar, double* __restrict__ mu) {
  const RowBlock b = blocks[blockIdx.x];
  int64_t row = b.row0 + threadIdx.x;
  if (row >= b.row1) return;
  for (int c = 0; c < nd; ++c) mu[row * nd + c] = rmask[row * nd + c] ? -rbar[b.sim] : 0.0;
}

// g on constrained unknowns -> 0 (the solve is over the free ones).
__global__ void k_mask(int64_t n, const uint8_t* __restrict__ cmask, double* __restrict__ v) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && cmask[k]) v[k] = 0.0;
}

// nu = mu - lambda (lambda is zero on constrained unknowns).
__global__ void k_nu(int64_t n, const double* __restrict__ mu, const double* __restrict__ lam, double* __restrict__ nu) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) nu[k] = mu[k] - lam[k];
}

// Per-sim sums of the per-particle parameter adjoints (sorted particles of a
// sim are contiguous: [p_begin, p_end)); one workgroup per sim, fixed order.
__global__ void __launch_bounds__(256) k_theta_sum(const SimDev* __restrict__ sims, int64_t np,
                                                  const double* __restrict__ theta_p, double* __restrict__ out) {
  const SimDev& S = sims[blockIdx.x];
  __shared__ double sh[2][4];
  for (int k = 0; k < 2; ++k) {
    double acc = 0.0;
    for (int64_t i = S.p_begin + threadIdx.x; i < S.p_end; i += 256) acc += theta_p[k * np + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = acc;
  }
  __syncthreads();
  if (threadIdx.x < 2) out[blockIdx.x * 2 + threadIdx.x] = (sh[threadIdx.x][0] + sh[threadIdx.x][1]) +
                                                            (sh[threadIdx.x][2] + sh[threadIdx.x][3]);
}

// Position of the transposed block: tpos[k] for block k = (r, c) is the index
// of block (c, r) (the pattern is structurally symmetric).
__global__ void k_tpos(int64_t n_row, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                       int32_t* __restrict__ tpos) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_row) return;
  for (int32_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
    int32_t c = colind[k];
    int32_t lo = rowptr[c], hi = rowptr[c + 1] - 1;
    while (lo < hi) {
      int32_t mid = (lo + hi) >> 1;
      if (colind[mid] < r) lo = mid + 1; else hi = mid;
    }
    tpos[k] = lo;
  }
}

// Transposed block-Jacobi inverse: D^-T.
__global__ void k_transpose_blocks(int64_t n, int bs, const double* __restrict__ in, double* __restrict__ out) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int i = 0; i < bs; ++i)
    for (int j = 0; j < bs; ++j) out[r * bs * bs + i * bs + j] = in[r * bs * bs + j * bs + i];
}

}  // namespace mpm

using namespace mpm;

int launch_tpos(mpm_ctx* c) {
  if (c->tpos_ready) return MPM_OK;
  if (c->tpos.ensure(c->nnzb) != hipSuccess) return c->fail(MPM_E_NOMEM, "tpos allocation failed");
  if (c->n_row) {
    k_tpos<<<(unsigned)((c->n_row + 255) / 256), 256, 0, c->stream>>>(c->n_row, c->rowptr.p, c->colind.p, c->tpos.p);
    LAUNCH_CHECK(c, "k_tpos");
  }
  c->tpos_ready = true;
  return MPM_OK;
}

extern "C" int mpm_adjoint_step(mpm_ctx* c, const mpm_problem* pb, const double* du, const double* react_bar,
                                const double* sbar_next, double* sbar_n, double* theta_bar, double krylov_rtol,
                                int32_t* krylov_iters, double* krylov_rel) {
  if (!c) return MPM_E_INVALID;
  c->err.clear();
  int rc = check_prepared(c, pb);
  if (rc) return rc;
  if (c->dim != 2 || c->up) return c->fail(MPM_E_INVALID, "the adjoint step covers plane-strain single-phase problems");
  if (pb->mat.shape != 0 || (pb->mat.dp && (pb->mat.dp_match & 3) == 3))
    return c->fail(MPM_E_INVALID, "the adjoint step covers B-spline Hencky, Drucker-Prager and Neo-Hookean problems");
  if (!du || !react_bar || !theta_bar) return c->fail(MPM_E_INVALID, "du, react_bar and theta_bar are required");
  HIPC(c, hipSetDevice(c->device));
  const int nd = c->nd, nsim = c->nsim;
  const int64_t nv = c->n_row * nd, np = c->np;
  bool ok = c->val.ensure(c->nnzb * nd * nd) == hipSuccess && c->kb.ensure(nv) == hipSuccess &&
            c->adj_mu.ensure(nv) == hipSuccess && c->adj_nu.ensure(nv) == hipSuccess &&
            c->adj_theta.ensure(2 * std::max<int64_t>(np, 1)) == hipSuccess &&
            c->adj_rbar.ensure(nsim) == hipSuccess && c->dinvT.ensure(c->n_row * nd * nd) == hipSuccess;
  if (!ok) return c->fail(MPM_E_NOMEM, "adjoint allocation failed");
  AdjArgs A;
  A.np = np; A.nd = nd; A.dp = c->dp; A.match = pb->mat.dp_match;
  A.xs = c->xs.p; A.vs = c->vol0s.p; A.Fs = c->Fs.p; A.bes = c->bes.p;
  A.Es = pb->P.E ? c->Es.p : nullptr; A.phis = pb->P.phi ? c->phis.p : nullptr;
  A.psim = c->psim.p; A.perm = c->perm.p; A.sims = c->sims.p; A.node_map = c->node_map.p; A.fp_user = pb->P.fp;
  A.E = pb->mat.E; A.nu = pb->mat.nu; A.phi = pb->mat.phi; A.c = pb->mat.c; A.psi = pb->mat.psi;
  A.apex_reg = pb->mat.apex_reg; A.rho0 = pb->mat.rho0;
  for (int k = 0; k < 3; ++k) A.g[k] = pb->mat.g[k];

  const unsigned nbk = (unsigned)c->blocks_h.size();
  const unsigned gv = (unsigned)std::max<int64_t>(1, (nv + 255) / 256);
  const unsigned gp = (unsigned)std::max<int64_t>(1, (np + 127) / 128);
  HIPC(c, hipMemcpyAsync(c->adj_rbar.p, react_bar, nsim * sizeof(double), hipMemcpyHostToDevice, c->stream));
  if (nbk) {
    k_adj_mu<<<nbk, 64, 0, c->stream>>>(c->blocks.p, nd, c->rmask.p, c->adj_rbar.p, c->adj_mu.p);
    LAUNCH_CHECK(c, "k_adj_mu");
  }
  // pass 1: g (into kb, the right-hand side of the transposed solve)
  HIPC(c, hipMemsetAsync(c->kb.p, 0, nv * sizeof(double), c->stream));
  if (np) {
    k_adj_g2<<<gp, 128, 0, c->stream>>>(A, du, c->adj_mu.p, sbar_next, c->kb.p);
    LAUNCH_CHECK(c, "k_adj_g2");
  }
  k_mask<<<gv, 256, 0, c->stream>>>(nv, c->cmask.p, c->kb.p);
  LAUNCH_CHECK(c, "k_mask");
  // J^T lambda = g with the step's Dirichlet-modified Jacobian
  rc = launch_jacobian(c, pb, du, c->val.p, true);
  if (rc) return rc;
  rc = launch_bj_inv(c, c->val.p);
  if (rc) return rc;
  rc = launch_tpos(c);
  if (rc) return rc;
  if (c->n_row) {
    k_transpose_blocks<<<(unsigned)((c->n_row + 255) / 256), 256, 0, c->stream>>>(c->n_row, nd, c->dinv.p,
                                                                                  c->dinvT.p);
    LAUNCH_CHECK(c, "k_transpose_blocks");
  }
  std::vector<int> kit;
  c->ktrans = true;
  c->kmethod = 0;
  const double artol = krylov_rtol > 0 ? krylov_rtol : 1e-12;
  rc = krylov_solve(c, c->val.p, artol, 20000, kit);
  c->ktrans = false;
  if (rc) return rc;
  if (krylov_iters)
    for (int s = 0; s < nsim; ++s) krylov_iters[s] = kit[s];
  if (krylov_rel)
    for (int s = 0; s < nsim; ++s) krylov_rel[s] = s < (int)c->kratio.size() ? c->kratio[s] : 0.0;
  if (c->krylov_soft) {
    // the Newton driver may continue from a stalled solve; a gradient may not
    double worst = 0.0;
    int ws = 0;
    for (int s = 0; s < (int)c->kratio.size(); ++s)
      if (c->kratio[s] > worst) { worst = c->kratio[s]; ws = s; }
    return c->fail(MPM_E_KRYLOV, "transposed solve stalled at true relative residual " + std::to_string(worst) +
                                     " (sim " + std::to_string(ws) + ") above krylov_rtol " + std::to_string(artol));
  }
  k_nu<<<gv, 256, 0, c->stream>>>(nv, c->adj_mu.p, c->kx.p, c->adj_nu.p);
  LAUNCH_CHECK(c, "k_nu");
  // pass 2: state and parameter adjoints
  if (np) {
    k_adj_s2<<<gp, 128, 0, c->stream>>>(A, du, c->adj_nu.p, sbar_next, sbar_n, c->adj_theta.p);
    LAUNCH_CHECK(c, "k_adj_s2");
  }
  k_theta_sum<<<nsim, 256, 0, c->stream>>>(c->sims.p, np, c->adj_theta.p, theta_bar);
  LAUNCH_CHECK(c, "k_theta_sum");
  return MPM_OK;
}
