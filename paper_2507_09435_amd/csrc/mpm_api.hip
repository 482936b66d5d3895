// C ABI entry points: argument validation, the Newton driver and dispatch.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "mpm_internal.hpp"

using namespace mpm;

namespace mpm {
__global__ void k_set_bc(int64_t nv, const uint8_t* __restrict__ cmask, const double* __restrict__ cval,
                         double* __restrict__ du) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nv && cmask[k]) du[k] = cval[k];
}
// b = -r on the rows of sims still iterating, 0 elsewhere.
__global__ void k_rhs(const RowBlock* __restrict__ blocks, int nd, const uint8_t* __restrict__ active,
                      const double* __restrict__ r, double* __restrict__ b) {
  const RowBlock blk = blocks[blockIdx.x];
  int64_t row = blk.row0 + threadIdx.x;
  if (row >= blk.row1) return;
  bool on = active[blk.sim] != 0;
  for (int c = 0; c < nd; ++c) b[row * nd + c] = on ? -r[row * nd + c] : 0.0;
}
__global__ void k_axpy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) y[k] += a * x[k];
}
// du = base + alpha[sim] * x per row block (line-search trial).
__global__ void k_trial(const RowBlock* __restrict__ blocks, int nd, const double* __restrict__ alpha,
                        const double* __restrict__ base, const double* __restrict__ x, double* __restrict__ du) {
  const RowBlock blk = blocks[blockIdx.x];
  int64_t row = blk.row0 + threadIdx.x;
  if (row >= blk.row1) return;
  double a = alpha[blk.sim];
  for (int c = 0; c < nd; ++c) du[row * nd + c] = base[row * nd + c] + a * x[row * nd + c];
}
}  // namespace mpm

// Scratch of mpm_residual_noalloc: the residual's per-particle force records
// in a fixed device array, so that call allocates nothing.  Each device the
// library runs on holds its own copy for the life of the process; host code
// reaches it only through the address hipGetSymbolAddress returns on that
// device (noalloc_scratch_ptr), never through the symbol itself.
static __device__ __align__(256) double scratch[MPM_NOALLOC_SCRATCH_BYTES / sizeof(double)];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MPM_MAX_DEVICES] = {};

// Called with `device` current (mpm_create).
static int noalloc_scratch_setup(int device) {
  if (device < 0 || device >= MPM_MAX_DEVICES) return MPM_E_INVALID;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return MPM_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MPM_E_HIP;
  g_scratch_ptr[device] = ptr;
  return MPM_OK;
}

static double* noalloc_scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < MPM_MAX_DEVICES) ? (double*)g_scratch_ptr[device] : nullptr;
}

int validate_problem(mpm_ctx* c, const mpm_problem* pb) {
  if (!pb) return c->fail(MPM_E_INVALID, "problem is NULL");
  if (pb->nsim < 1) return c->fail(MPM_E_INVALID, "nsim must be >= 1");
  if (!pb->grids) return c->fail(MPM_E_INVALID, "grids is NULL");
  if (pb->nsim > 1 && !pb->sim_start) return c->fail(MPM_E_INVALID, "sim_start is required for nsim > 1");
  const int dim = pb->grids[0].dim;
  if (dim != 2 && dim != 3) return c->fail(MPM_E_INVALID, "dim must be 2 or 3");
  if (pb->mat.up && dim != 2) return c->fail(MPM_E_INVALID, "u-p is available in plane strain only");
  for (int s = 0; s < pb->nsim; ++s) {
    const mpm_grid& g = pb->grids[s];
    if (g.dim != dim) return c->fail(MPM_E_INVALID, "all sims of a batch must share dim");
    if (!(g.h > 0.0) || !std::isfinite(g.h)) return c->fail(MPM_E_INVALID, "grid spacing must be positive");
    for (int k = 0; k < dim; ++k)
      if (g.ncell[k] < 1 || g.ncell[k] > (1 << 20)) return c->fail(MPM_E_INVALID, "ncell out of range");
  }
  const int64_t np = pb->P.np;
  if (np < 0 || np >= (int64_t)INT32_MAX) return c->fail(MPM_E_INVALID, "np out of range");
  if (np > 0 && (!pb->P.x || !pb->P.vol0 || !pb->P.F || !pb->P.be))
    return c->fail(MPM_E_INVALID, "particle arrays x, vol0, F, be are required");
  if (!pb->bc_mask || !pb->bc_value) return c->fail(MPM_E_INVALID, "bc_mask and bc_value are required");
  if (pb->sim_start) {
    if (pb->sim_start[0] != 0 || pb->sim_start[pb->nsim] != np)
      return c->fail(MPM_E_INVALID, "sim_start must run from 0 to np");
    for (int s = 0; s < pb->nsim; ++s)
      if (pb->sim_start[s + 1] < pb->sim_start[s]) return c->fail(MPM_E_INVALID, "sim_start must be non-decreasing");
  }
  if (!(pb->mat.E > 0.0) && !pb->P.E) return c->fail(MPM_E_INVALID, "Young's modulus must be positive");
  if (!(pb->mat.nu > -1.0 && pb->mat.nu < 0.5)) return c->fail(MPM_E_INVALID, "Poisson ratio out of range");
  if ((pb->mat.dp_match & ~7) != 0)
    return c->fail(MPM_E_INVALID, "dp_match must be 0, 1, 2 or 3, plus 4 for associated flow");
  if ((pb->mat.dp_match & 3) == 3 && pb->mat.dp && !(pb->mat.c > 0.0))
    return c->fail(MPM_E_INVALID, "J2 plasticity (dp_match 3) needs a positive yield strength c");
  if (pb->mat.shape != 0 && pb->mat.shape != 1) return c->fail(MPM_E_INVALID, "shape must be 0 or 1");
  if (pb->mat.elastic != 0 && pb->mat.elastic != 1) return c->fail(MPM_E_INVALID, "elastic must be 0 or 1");
  if (pb->mat.elastic == 1 && pb->mat.dp)
    return c->fail(MPM_E_INVALID, "the Neo-Hookean law is elastic (dp must be 0)");
  if (pb->mat.shape == 1)
    for (int k = 0; k < dim; ++k)
      if (!(pb->mat.lp0[k] > 0.0)) return c->fail(MPM_E_INVALID, "cpGIMP needs lp0 > 0 on every axis");
  return MPM_OK;
}

int check_prepared(mpm_ctx* c, const mpm_problem* pb) {
  if (!pb) return c->fail(MPM_E_INVALID, "problem is NULL");
  if (!c->prepared) return c->fail(MPM_E_INVALID, "mpm_prepare has not run (or failed) for this problem");
  if (pb->P.np != c->np || pb->P.x != c->user_x || pb->nsim != c->nsim || !pb->grids || pb->grids[0].dim != c->dim ||
      (pb->mat.up ? 1 : 0) != c->up)
    return c->fail(MPM_E_INVALID, "problem differs from the one given to mpm_prepare");
  return MPM_OK;
}

// Device buffers of a context and of its multigrid levels.
void ctx_release(mpm_ctx* c) {
  mg_release(c);
  c->sims.release(); c->sim_start.release(); c->okey.release(); c->gcount.release(); c->gstart.release();
  c->cursor.release(); c->okey_sorted.release(); c->sort_hist.release(); c->sort_off.release(); c->perm.release(); c->psim.release(); c->scan_tmp.release(); c->node_flag.release();
  c->node_map.release(); c->active_nodes.release(); c->row_sim.release(); c->rowcnt.release(); c->rowptr.release();
  c->colind.release(); c->slot.release(); c->rgrp.release(); c->bcode.release(); c->blocks.release(); c->blk_first.release(); c->flag.release();
  c->xs.release(); c->vol0s.release(); c->Fs.release(); c->bes.release(); c->Es.release(); c->phis.release();
  c->cmask.release(); c->rmask.release(); c->cval.release(); c->fext.release(); c->fint.release(); c->nvol.release();
  c->work.release(); c->val.release(); c->dinv.release(); c->pdat.release(); c->pdat3.release(); c->pdF3.release(); c->jc3_ws.release(); c->jl3_ws.release(); c->jf3_ws.release(); c->gbuf.release(); c->rrec.release();
  c->kx.release(); c->kr.release(); c->krh.release(); c->kp.release(); c->kv.release(); c->ks.release();
  c->kt.release(); c->kph.release(); c->ksh.release(); c->kb.release(); c->part.release(); c->simsc.release();
  c->simflag.release(); c->du_base.release(); c->alpha.release();
  c->gV.release(); c->gsc.release(); c->gpart.release(); c->gflag.release(); c->greset.release();
  c->tpos.release(); c->dinvT.release(); c->adj_mu.release(); c->adj_nu.release(); c->adj_theta.release();
  c->adj_rbar.release();
}

extern "C" {

int mpm_create(mpm_ctx** out, int device, void* stream) {
  if (!out) return MPM_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MPM_E_INVALID;
  if (hipSetDevice(device) != hipSuccess) return MPM_E_HIP;
  if (device >= MPM_MAX_DEVICES) return MPM_E_INVALID;
  const int src = noalloc_scratch_setup(device);
  if (src) return src;
  mpm_ctx* c = new (std::nothrow) mpm_ctx();
  if (!c) return MPM_E_NOMEM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  *out = c;
  return MPM_OK;
}

int mpm_destroy(mpm_ctx* c) {
  if (!c) return MPM_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  ctx_release(c);
  delete c;
  return MPM_OK;
}

const char* mpm_last_error(const mpm_ctx* c) { return c ? c->err.c_str() : "null context"; }

int mpm_prepare(mpm_ctx* c, const mpm_problem* pb, int64_t* n_row, int64_t* nnzb, int32_t* nd) {
  if (!c) return MPM_E_INVALID;
  c->err.clear();
  HIPC(c, hipSetDevice(c->device));
  return mpm_prepare_impl(c, pb, n_row, nnzb, nd);
}

int mpm_residual(mpm_ctx* c, const mpm_problem* pb, const double* du, double* r, double* r_raw, double* reaction) {
  if (!c) return MPM_E_INVALID;
  c->err.clear();
  GUARD(check_prepared(c, pb));
  if (!du && c->n_row) return c->fail(MPM_E_INVALID, "du is NULL");
  HIPC(c, hipSetDevice(c->device));
  GUARD(launch_residual(c, pb, du, r, r_raw));
  if (reaction) {
    std::vector<double> sc(16 * c->nsim);
    HIPC(c, hipMemcpyAsync(sc.data(), c->simsc.p, sc.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPC(c, hipStreamSynchronize(c->stream));
    for (int s = 0; s < c->nsim; ++s) reaction[s] = -sc[s * 16 + 1];
  }
  return MPM_OK;
}

int mpm_residual_noalloc(mpm_ctx* c, const mpm_problem* pb, const double* du, double* r, double* r_raw,
                         double* reaction) {
  if (!c) return MPM_E_INVALID;
  c->err.clear();
  GUARD(check_prepared(c, pb));
  if (!du && c->n_row) return c->fail(MPM_E_INVALID, "du is NULL");
  const int64_t need = c->np * fint_record_doubles(c->dim) * (int64_t)sizeof(double);
  if (need > (int64_t)MPM_NOALLOC_SCRATCH_BYTES)
    return c->fail(MPM_E_INVALID, "mpm_residual_noalloc: " + std::to_string(c->np) + " particles need " +
                                      std::to_string(need) + " bytes of scratch, more than its fixed " +
                                      std::to_string((long long)MPM_NOALLOC_SCRATCH_BYTES));
  HIPC(c, hipSetDevice(c->device));
  double* rec = noalloc_scratch_ptr(c->device);
  if (!rec) return c->fail(MPM_E_HIP, "scratch address of this device is not set up");
  GUARD(launch_residual(c, pb, du, r, r_raw, rec));
  if (reaction) {
    // column 1 of the per-sim scalars [nsim][16], straight into the caller's array
    HIPC(c, hipMemcpy2DAsync(reaction, sizeof(double), c->simsc.p + 1, 16 * sizeof(double), sizeof(double),
                             c->nsim, hipMemcpyDeviceToHost, c->stream));
    HIPC(c, hipStreamSynchronize(c->stream));
    for (int s = 0; s < c->nsim; ++s) reaction[s] = -reaction[s];
  }
  return MPM_OK;
}

int mpm_jacobian_bsr(mpm_ctx* c, const mpm_problem* pb, const double* du, int32_t* rowptr, int32_t* colind,
                     double* val, int64_t* active_nodes, int32_t flags) {
  if (!c) return MPM_E_INVALID;
  c->err.clear();
  GUARD(check_prepared(c, pb));
  HIPC(c, hipSetDevice(c->device));
  if (rowptr)
    HIPC(c, hipMemcpyAsync(rowptr, c->rowptr.p, (c->n_row + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
  if (colind && c->nnzb)
    HIPC(c, hipMemcpyAsync(colind, c->colind.p, c->nnzb * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
  if (active_nodes && c->n_row)
    HIPC(c, hipMemcpyAsync(active_nodes, c->active_nodes.p, c->n_row * sizeof(int64_t), hipMemcpyDeviceToDevice,
                           c->stream));
  if (val) {
    if (!du && c->n_row) return c->fail(MPM_E_INVALID, "du is NULL");
    GUARD(launch_jacobian(c, pb, du, val, (flags & MPM_JAC_RAW) == 0));
  }
  return MPM_OK;
}

int mpm_jv(mpm_ctx* c, const mpm_problem* pb, const double* du, const double* x, double* y, int32_t flags) {
  if (!c) return MPM_E_INVALID;
  c->err.clear();
  GUARD(check_prepared(c, pb));
  if (c->n_row && (!x || !y)) return c->fail(MPM_E_INVALID, "x and y are required");
  const bool reuse = (flags & MPM_JV_REUSE) != 0;
  if (!reuse && !du && c->n_row) return c->fail(MPM_E_INVALID, "du is NULL");
  if (x == y && c->n_row) return c->fail(MPM_E_INVALID, "x and y must not alias");
  HIPC(c, hipSetDevice(c->device));
  if (!reuse) HIPC(c, hipMemsetAsync(c->flag.p, 0, sizeof(int32_t), c->stream));
  return launch_jv(c, pb, du, !reuse, x, y, (flags & MPM_JAC_RAW) == 0);
}

int mpm_update(mpm_ctx* c, const mpm_problem* pb, const double* du, double* x_out, double* F_out, double* be_out) {
  if (!c) return MPM_E_INVALID;
  c->err.clear();
  GUARD(check_prepared(c, pb));
  if (!du && c->n_row) return c->fail(MPM_E_INVALID, "du is NULL");
  HIPC(c, hipSetDevice(c->device));
  HIPC(c, hipMemsetAsync(c->flag.p, 0, sizeof(int32_t), c->stream));
  GUARD(launch_update(c, pb, du, x_out, F_out, be_out));
  if ((x_out && x_out == pb->P.x) || (F_out && F_out == pb->P.F) || (be_out && be_out == pb->P.be))
    c->prepared = false;   // the problem's state has moved past the one prepare sorted
  int32_t hf = 0;
  HIPC(c, hipMemcpyAsync(&hf, c->flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  if (hf & 4) return c->fail(MPM_E_RANGE, "elastic strain outside the log series range");
  return MPM_OK;
}

int mpm_newton_step(mpm_ctx* c, const mpm_problem* pb, const mpm_newton_opts* opts, double* du,
                    mpm_newton_report* rep) {
  if (!c) return MPM_E_INVALID;
  c->err.clear();
  GUARD(check_prepared(c, pb));
  if (!opts || (!du && c->n_row)) return c->fail(MPM_E_INVALID, "du and opts are required");
  if (!(opts->tol > 0.0) || opts->max_iter < 0 || opts->max_iter > 1000)
    return c->fail(MPM_E_INVALID, "Newton options out of range");
  HIPC(c, hipSetDevice(c->device));
  const int nsim = c->nsim, nd = c->nd;
  const int64_t nv = c->n_row * nd;
  const double rtol_fixed = opts->krylov_rtol;
  const int kmax = opts->krylov_max_iter > 0 ? opts->krylov_max_iter : 20000;
  if (opts->krylov_method < 0 || opts->krylov_method > 3) return c->fail(MPM_E_INVALID, "unknown krylov_method");
  const bool use_mg = opts->krylov_method >= 2;
  c->kmethod = opts->krylov_method;
  if (use_mg && !c->mg_ready) GUARD(mg_build(c, pb));
  const double stall = opts->stall_factor > 0 ? opts->stall_factor : 0.0;
  if (c->val.ensure(c->nnzb * nd * nd) != hipSuccess || c->kb.ensure(nv) != hipSuccess ||
      c->work.ensure(nv) != hipSuccess)
    return c->fail(MPM_E_NOMEM, "Newton allocation failed");
  DBuf<uint8_t> active;
  if (active.ensure(nsim) != hipSuccess) return c->fail(MPM_E_NOMEM, "Newton allocation failed");
  struct Release { DBuf<uint8_t>& a; ~Release() { a.release(); } } rel{active};

  hipEvent_t ev[8];
  for (int k = 0; k < 8; ++k) HIPC(c, hipEventCreate(&ev[k]));
  struct EvRelease { hipEvent_t* e; ~EvRelease() { for (int k = 0; k < 8; ++k) (void)hipEventDestroy(e[k]); } } erel{ev};
  float ms_res = 0, ms_jac = 0, ms_kry = 0;
  c->time_spmv = opts->time_spmv > 0 ? opts->time_spmv : 0;
  c->spmv_ms = 0.0;
  c->spmv_n = 0;
  HIPC(c, hipEventRecord(ev[6], c->stream));

  unsigned g = (unsigned)std::max<int64_t>(1, (nv + 255) / 256);
  k_set_bc<<<g, 256, 0, c->stream>>>(nv, c->cmask.p, c->cval.p, du);
  HIPC(c, hipMemsetAsync(c->flag.p, 0, sizeof(int32_t), c->stream));
  LAUNCH_CHECK(c, "k_set_bc");

  std::vector<double> norm0(nsim, -1.0), prev(nsim, -1.0), react(nsim, 0.0), sc(16 * nsim);
  std::vector<int> conv(nsim, 0), iters(nsim, 0);
  std::vector<uint8_t> act(nsim, 1);
  std::vector<int> kit;
  int64_t kr_total = 0;
  int it = 0, status = MPM_OK;
  if (rep) {
    rep->iters = 0; rep->converged = 0; rep->krylov_iters = 0;
    for (int k = 0; k < MPM_MAX_REPORT; ++k) { rep->norms[k] = 0.0; rep->krylov[k] = 0; }
  }
  for (it = 0;; ++it) {
    HIPC(c, hipEventRecord(ev[0], c->stream));
    GUARD(launch_residual(c, pb, du, c->work.p, nullptr));
    HIPC(c, hipEventRecord(ev[1], c->stream));
    HIPC(c, hipMemcpyAsync(sc.data(), c->simsc.p, 16 * nsim * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPC(c, hipStreamSynchronize(c->stream));
    float t = 0;
    HIPC(c, hipEventElapsedTime(&t, ev[0], ev[1]));
    ms_res += t;
    bool all = true;
    for (int s = 0; s < nsim; ++s) {
      double nrm = std::sqrt(sc[s * 16 + 0]);
      if (!std::isfinite(nrm)) return c->fail(MPM_E_NONFINITE, "residual norm is not finite");
      if (conv[s]) continue;
      if (norm0[s] < 0) norm0[s] = nrm;
      react[s] = -sc[s * 16 + 1];
      bool ok = nrm <= opts->tol * norm0[s] || nrm == 0.0;
      if (!ok && stall > 0 && prev[s] >= 0 && nrm <= stall * opts->tol * norm0[s] && nrm > 0.5 * prev[s]) ok = true;
      prev[s] = nrm;
      if (ok) { conv[s] = 1; iters[s] = it; act[s] = 0; }
      all = all && conv[s];
    }
    if (rep && it < MPM_MAX_REPORT) rep->norms[it] = std::sqrt(sc[0]);
    if (all) break;
    if (it >= opts->max_iter) { status = MPM_E_NOT_CONVERGED; break; }
    // Jacobian and linear solve for the sims still iterating
    HIPC(c, hipEventRecord(ev[2], c->stream));
    GUARD(launch_jacobian(c, pb, du, c->val.p, true));
    HIPC(c, hipEventRecord(ev[3], c->stream));
    // preconditioner setup belongs to the linear solve's time
    GUARD(launch_bj_inv(c, c->val.p));
    if (use_mg) GUARD(mg_setup(c));
    HIPC(c, hipMemcpyAsync(active.p, act.data(), nsim, hipMemcpyHostToDevice, c->stream));
    if (!c->blocks_h.empty()) {
      k_rhs<<<(unsigned)c->blocks_h.size(), 64, 0, c->stream>>>(c->blocks.p, nd, active.p, c->work.p, c->kb.p);
      LAUNCH_CHECK(c, "k_rhs");
    }
    double rtol = rtol_fixed > 0 ? rtol_fixed : 1e-12;
    int rc = krylov_solve(c, c->val.p, rtol, kmax, kit);
    HIPC(c, hipEventRecord(ev[4], c->stream));
    int64_t kmx = 0;
    for (int s = 0; s < nsim; ++s) { kr_total += kit[s]; kmx = std::max<int64_t>(kmx, kit[s]); }
    if (rep && it < MPM_MAX_REPORT) rep->krylov[it] = (int32_t)kmx;
    if (rc) { status = rc; break; }
    if (opts->line_search > 0 && !c->blocks_h.empty()) {
      // backtracking per sim on the residual norm
      if (c->du_base.ensure(nv) != hipSuccess || c->alpha.ensure(nsim) != hipSuccess)
        return c->fail(MPM_E_NOMEM, "line-search allocation failed");
      HIPC(c, hipMemcpyAsync(c->du_base.p, du, nv * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      std::vector<double> alpha(nsim, 1.0);
      std::vector<int> done(nsim, 0);
      for (int s = 0; s < nsim; ++s) if (!act[s]) { alpha[s] = 0.0; done[s] = 1; }
      const unsigned nbk = (unsigned)c->blocks_h.size();
      // step lengths 1, 1/2, ..., 2^-(L-1); a sim that finds no decrease in
      // those L trials takes the full step
      bool fallback = false;
      for (int trial = 0; trial < opts->line_search; ++trial) {
        HIPC(c, hipMemcpyAsync(c->alpha.p, alpha.data(), nsim * sizeof(double), hipMemcpyHostToDevice, c->stream));
        k_trial<<<nbk, 64, 0, c->stream>>>(c->blocks.p, nd, c->alpha.p, c->du_base.p, c->kx.p, du);
        LAUNCH_CHECK(c, "k_trial");
        GUARD(launch_residual(c, pb, du, c->work.p, nullptr));
        HIPC(c, hipMemcpyAsync(sc.data(), c->simsc.p, 16 * nsim * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPC(c, hipStreamSynchronize(c->stream));
        bool pending = false;
        for (int s = 0; s < nsim; ++s) {
          if (done[s]) continue;
          double nt = std::sqrt(sc[s * 16 + 0]);
          if (std::isfinite(nt) && nt < (1.0 - 1e-4 * alpha[s]) * prev[s]) { done[s] = 1; continue; }
          if (trial + 1 == opts->line_search) { alpha[s] = 1.0; done[s] = 1; fallback = true; continue; }
          alpha[s] *= 0.5;
          pending = true;
        }
        if (!pending) break;
      }
      if (fallback) {   // du still holds the last trial: rebuild it with the final step lengths
        HIPC(c, hipMemcpyAsync(c->alpha.p, alpha.data(), nsim * sizeof(double), hipMemcpyHostToDevice, c->stream));
        k_trial<<<nbk, 64, 0, c->stream>>>(c->blocks.p, nd, c->alpha.p, c->du_base.p, c->kx.p, du);
        LAUNCH_CHECK(c, "k_trial");
      }
    } else {
      k_axpy<<<g, 256, 0, c->stream>>>(nv, 1.0, c->kx.p, du);
      LAUNCH_CHECK(c, "k_axpy");
    }
    HIPC(c, hipEventRecord(ev[5], c->stream));
    HIPC(c, hipEventSynchronize(ev[5]));
    HIPC(c, hipEventElapsedTime(&t, ev[2], ev[3]));
    ms_jac += t;
    HIPC(c, hipEventElapsedTime(&t, ev[3], ev[4]));
    ms_kry += t;
  }
  int32_t hf = 0;
  HIPC(c, hipMemcpyAsync(&hf, c->flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  if (status == MPM_E_KRYLOV && (hf & 24)) {
    std::string why;
    if (hf & 8) why += " a singular or missing diagonal block was replaced by the identity in block-Jacobi;";
    if (hf & 16) why += " a zero pivot in the coarsest multigrid solve left a column unreduced;";
    c->err += " (preconditioner faults:" + why + ")";
  }
  if (status == MPM_OK && (hf & 4)) status = c->fail(MPM_E_RANGE, "elastic strain outside the log series range");
  if (status == MPM_OK && opts->commit) {
    GUARD(launch_update(c, pb, du, pb->P.x, pb->P.F, pb->P.be));
    c->prepared = false;   // the sorted copies hold the step-start state, the caller's arrays the new one
  }
  HIPC(c, hipEventRecord(ev[7], c->stream));
  HIPC(c, hipEventSynchronize(ev[7]));
  float tt = 0;
  HIPC(c, hipEventElapsedTime(&tt, ev[6], ev[7]));
  int itmax = 0;
  bool allc = true;
  for (int s = 0; s < nsim; ++s) {
    if (!conv[s]) iters[s] = it;
    itmax = std::max(itmax, iters[s]);
    allc = allc && conv[s];
  }
  if (rep) {
    rep->iters = itmax;
    rep->converged = allc ? 1 : 0;
    rep->krylov_iters = kr_total;
    rep->ms_residual = ms_res; rep->ms_jacobian = ms_jac; rep->ms_krylov = ms_kry; rep->ms_total = tt;
    rep->spmv_ms = c->spmv_ms; rep->spmv_launches = c->spmv_n;
    rep->precond_flags = hf & 24;
    for (int s = 0; s < nsim; ++s) {
      if (rep->sim_iters) rep->sim_iters[s] = iters[s];
      if (rep->sim_converged) rep->sim_converged[s] = conv[s];
      if (rep->sim_reaction) rep->sim_reaction[s] = react[s];
      if (rep->sim_rel) rep->sim_rel[s] = norm0[s] > 0 ? prev[s] / norm0[s] : 0.0;
    }
  }
  c->time_spmv = 0;
  if (status == MPM_E_NOT_CONVERGED) return c->fail(MPM_E_NOT_CONVERGED, "Newton did not converge");
  return status;
}

int mpm_spmv_lanes(const mpm_ctx* c) { return c ? c->spmv_lanes : 0; }

int mpm_spmv_set_lanes(mpm_ctx* c, int32_t lanes) {
  if (!c) return MPM_E_INVALID;
  c->err.clear();
  if (lanes != 0 && lanes != 4 && lanes != 8 && lanes != 16)
    return c->fail(MPM_E_INVALID, "lanes per row must be 0, 4, 8 or 16");
  c->spmv_pin = lanes;
  c->spmv_lanes = lanes;
  return MPM_OK;
}

int mpm_spmv(mpm_ctx* c, const double* val, const double* x, double* y, const double* z) {
  if (!c) return MPM_E_INVALID;
  c->err.clear();
  if (!c->prepared) return c->fail(MPM_E_INVALID, "mpm_prepare has not run");
  if (!val || !x || !y || x == y || z == y) return c->fail(MPM_E_INVALID, "val, x, y are required; y must not alias x or z");
  HIPC(c, hipSetDevice(c->device));
  return launch_spmv(c, val, x, y, z);
}

}  // extern "C"
