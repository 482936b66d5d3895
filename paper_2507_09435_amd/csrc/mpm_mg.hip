// Geometric multigrid preconditioner for the 2-D single-phase Newton
// systems (the GPU counterpart of the algebraic multigrid the paper uses
// on the CPU, Remark 2).
//
// Levels: level l is the same set of particles on a grid of cell size
// 2^l h (ceil(n / 2^l) cells per axis, same origin).  Its operator is
// assembled like the fine Jacobian, from the particles' tangent tables at the
// current Newton iterate contracted with the level's own B-spline gradients
// (Sec. 3.2's local blocks on a coarser background grid), so no Galerkin
// product is formed.  A coarse node is constrained where the fine node at
// the same position is.  Transfers: linear interpolation between node
// lattices (fine node 2I takes coarse node I, an odd fine node the mean of
// its two coarse neighbours); restriction is its transpose, as a gather.
// Smoother: damped block-Jacobi.  Coarsest level: per-simulation dense
// inverse (Gauss-Jordan with partial pivoting on the device).
//
// One V-cycle is a fixed linear map, so it serves as the right
// preconditioner of BiCGStab.
#include "mpm_internal.hpp"

namespace mpm {

constexpr int MG_NU1 = 2, MG_NU2 = 2;   // pre- and post-smoothing sweeps
constexpr double MG_OMEGA = 0.6;        // damping of the block-Jacobi sweeps
constexpr int MG_MAX_LEVELS = 12;
constexpr int MG_DENSE_MAX = 64;        // coarsest unknowns per simulation (inverted in LDS)
constexpr int MG_TAIL_ROWS = 256;       // levels with at most this many rows per sim run in one launch

// Multiply-adds of the V-cycle are written as explicit fma with a fixed
// operand order: left to contraction, the compiler may fuse a different
// product of the same expression in different kernels, and the fused tail,
// the fused first sweep and the level-by-level launches must round alike.
__device__ __forceinline__ double dot2(double a0, double x0, double a1, double x1) { return fma(a0, x0, a1 * x1); }

__device__ __forceinline__ int sim_of_node(const SimDev* sims, int nsim, int64_t node) {
  int s = 0;
  while (s + 1 < nsim && node >= sims[s + 1].node_base) ++s;
  return s;
}

// Coarse full-grid mask from the next finer one (same node position).
__global__ void k_mg_mask(int64_t n_cnodes, int nsim, const SimDev* __restrict__ csims,
                          const SimDev* __restrict__ fsims, const uint8_t* __restrict__ fmask,
                          uint8_t* __restrict__ cmask) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_cnodes) return;
  const int s = sim_of_node(csims, nsim, g);
  const SimDev& C = csims[s];
  const SimDev& F = fsims[s];
  const int64_t loc = g - C.node_base;
  const int I = (int)(loc % C.nna[0]) - 1, J = (int)(loc / C.nna[0]) - 1;
  const int i = min(max(2 * I, -1), F.n[0] + 1), j = min(max(2 * J, -1), F.n[1] + 1);
  const int64_t fn = F.node_base + (i + 1) + (int64_t)F.nna[0] * (j + 1);
  cmask[g * 2 + 0] = fmask[fn * 2 + 0];
  cmask[g * 2 + 1] = fmask[fn * 2 + 1];
}

__global__ void k_mg_inv_perm(int64_t np, const int32_t* __restrict__ perm, int32_t* __restrict__ inv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) inv[perm[i]] = (int32_t)i;
}

__global__ void k_mg_pmap(int64_t np, const int32_t* __restrict__ perm, const int32_t* __restrict__ inv,
                          int32_t* __restrict__ pmap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) pmap[i] = inv[perm[i]];
}

// Level records: the finest record's tangent table, this level's weights.
__global__ void k_mg_rec2(int64_t np, const double* __restrict__ xs, const int32_t* __restrict__ psim,
                          const SimDev* __restrict__ sims, const int32_t* __restrict__ pmap,
                          const double* __restrict__ fpdat, double* __restrict__ cpdat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const double* F = fpdat + (int64_t)pmap[i] * PD2;
  double* C = cpdat + i * PD2;
#pragma unroll
  for (int k = 0; k < 16; ++k) C[k] = F[k];
  Stencil<2> st;
  make_stencil<2>(sims[psim[i]], xs, np, i, st);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C[16 + a] = st.w[0][a];
    C[19 + a] = st.dw[0][a];
    C[22 + a] = st.w[1][a];
    C[25 + a] = st.dw[1][a];
  }
}

// One block-Jacobi step on one row (LPR lanes per row):
// mode 0: x_out = w D^-1 b;  mode 1: x_out = x_in + w D^-1 (b - A x_in);
// mode 2: x_out = b - A x_in;  mode 3: modes 0 and 1 in one pass, the
// mode-0 iterate of each neighbour formed on the fly from its D^-1 and b
// with mode 0's own expression (so the same bits as the two passes).  The row product does not depend on LPR
// (2, 4 or 8): block k of the row adds into partial sum k mod 8 in ascending
// k, and the 8 partial sums meet in a fixed butterfly (offsets 4, 2, 1),
// the levels at offsets >= LPR inside the lane.
template <int LPR, int mode>
__device__ __forceinline__ void mg_sweep_row(int row, int lane, int k0r, int k1,
                                             const int32_t* __restrict__ colind, const double* __restrict__ val,
                                             const double* __restrict__ dinv, const double* __restrict__ b,
                                             const double* __restrict__ x_in, double* __restrict__ x_out,
                                             double omega) {
  constexpr int VL = 8, NA = VL / LPR;
  static_assert(NA == 1 || NA == 2 || NA == 4, "LPR must be 2, 4 or 8");
  double a0 = 0.0, a1 = 0.0;
  if (mode != 0) {
    double p0[NA], p1[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) p0[a] = p1[a] = 0.0;
    // four steps of VL blocks at a time: every index, block and x entry of
    // the batch is loaded before the first sum (indices past the row's end
    // read its last block and are not added), then the sums take the blocks
    // in the order of the one-step loop
    constexpr int NS = 4;
    for (int kb = k0r + lane; kb < k1; kb += NS * VL) {
      int64_t cc[NS][NA];
      double bl[NS][NA][4], xv[NS][NA][2];
#pragma unroll
      for (int j = 0; j < NS; ++j)
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          const int k = min(kb + j * VL + a * LPR, k1 - 1);
          cc[j][a] = colind[k];
#pragma unroll
          for (int e = 0; e < 4; ++e) bl[j][a][e] = val[(int64_t)k * 4 + e];
        }
      if (mode == 3) {
#pragma unroll
        for (int j = 0; j < NS; ++j)
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            const int64_t c = cc[j][a];
            const double* Dc = dinv + c * 4;
            const double s0 = b[c * 2], s1 = b[c * 2 + 1];
            xv[j][a][0] = fma(omega, dot2(Dc[0], s0, Dc[1], s1), 0.0);
            xv[j][a][1] = fma(omega, dot2(Dc[2], s0, Dc[3], s1), 0.0);
          }
      } else {
#pragma unroll
        for (int j = 0; j < NS; ++j)
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            xv[j][a][0] = x_in[cc[j][a] * 2];
            xv[j][a][1] = x_in[cc[j][a] * 2 + 1];
          }
      }
#pragma unroll
      for (int j = 0; j < NS; ++j)
#pragma unroll
        for (int a = 0; a < NA; ++a)
          if (kb + j * VL + a * LPR < k1) {
            p0[a] = p0[a] + dot2(bl[j][a][0], xv[j][a][0], bl[j][a][1], xv[j][a][1]);
            p1[a] = p1[a] + dot2(bl[j][a][2], xv[j][a][0], bl[j][a][3], xv[j][a][1]);
          }
    }
#pragma unroll
    for (int m = NA / 2; m > 0; m >>= 1)
#pragma unroll
      for (int a = 0; a < m; ++a) { p0[a] += p0[a + m]; p1[a] += p1[a + m]; }
    a0 = p0[0];
    a1 = p1[0];
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off, LPR);
      a1 += __shfl_xor(a1, off, LPR);
    }
  }
  if (lane == 0) {
    const double r0 = b[(int64_t)row * 2] - a0, r1 = b[(int64_t)row * 2 + 1] - a1;
    if (mode == 2) {
      x_out[(int64_t)row * 2] = r0;
      x_out[(int64_t)row * 2 + 1] = r1;
    } else {
      const double* D = dinv + (int64_t)row * 4;
      double base0 = mode == 1 ? x_in[(int64_t)row * 2] : 0.0;
      double base1 = mode == 1 ? x_in[(int64_t)row * 2 + 1] : 0.0;
      if (mode == 3) {   // this row's mode-0 iterate
        const double s0 = b[(int64_t)row * 2], s1 = b[(int64_t)row * 2 + 1];
        base0 = fma(omega, dot2(D[0], s0, D[1], s1), 0.0);
        base1 = fma(omega, dot2(D[2], s0, D[3], s1), 0.0);
      }
      x_out[(int64_t)row * 2] = fma(omega, dot2(D[0], r0, D[1], r1), base0);
      x_out[(int64_t)row * 2 + 1] = fma(omega, dot2(D[2], r0, D[3], r1), base1);
    }
  }
}

// One sweep over the rows of a level, 64 rows per workgroup in row order
// (a sweep has no per-block sums, so rows need not follow the row blocks).
// A row reads its sim beside its row pointers; rows of sims whose Krylov
// solve is finished (flag set) leave before their block loads, so a batch
// does no work for its finished sims.
template <int LPR, int mode>
__global__ void __launch_bounds__(ROWS_PER_BLOCK * LPR) k_mg_sweep(
    int64_t n_row, const int32_t* __restrict__ row_sim, const int32_t* __restrict__ simflag,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind, const double* __restrict__ val,
    const double* __restrict__ dinv, const double* __restrict__ b, const double* __restrict__ x_in,
    double* __restrict__ x_out, double omega) {
  const int lane = threadIdx.x % LPR, grp = threadIdx.x / LPR;
  const int64_t row = (int64_t)blockIdx.x * ROWS_PER_BLOCK + grp;
  if (row >= n_row) return;   // the row's LPR lanes leave together
  const int k0r = rowptr[row], k1r = rowptr[row + 1];
  if (simflag[2 * row_sim[row]] >= 0) return;   // the row's LPR lanes leave together
  mg_sweep_row<LPR, mode>((int)row, lane, k0r, k1r, colind, val, dinv, b, x_in, x_out, omega);
}

// The first post-smoothing sweep with the prolongation folded in: every
// value of the iterate it reads is x_in + P x_c (unconstrained unknowns),
// formed from the per-row prolongation table in the terms and order of the
// prolongation itself; then mode 1 of mg_sweep_row on those values.
__device__ __forceinline__ void mg_prolonged(int64_t r, const int32_t* __restrict__ ptab,
                                             const double* __restrict__ pw, const double* __restrict__ xc,
                                             const uint8_t* __restrict__ cmask, const double* __restrict__ x_in,
                                             double& x0, double& x1) {
  // the table lists its coarse rows first, then -1: every entry is loaded
  // at once (a -1 entry reads this row's own x_in, always in bounds, and is
  // not added) and the terms are added in table order
  int32_t cr[4];
  double v[4][2];
#pragma unroll
  for (int q = 0; q < 4; ++q) cr[q] = ptab[r * 4 + q];
  const double w = pw[r];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double* src = cr[q] >= 0 ? xc + (int64_t)cr[q] * 2 : x_in + r * 2;
    v[q][0] = src[0];
    v[q][1] = src[1];
  }
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (cr[q] >= 0) {
      a0 = fma(w, v[q][0], a0);
      a1 = fma(w, v[q][1], a1);
    }
  x0 = x_in[r * 2];
  x1 = x_in[r * 2 + 1];
  if (!cmask[r * 2]) x0 += a0;
  if (!cmask[r * 2 + 1]) x1 += a1;
}

template <int LPR>
__global__ void __launch_bounds__(ROWS_PER_BLOCK * LPR) k_mg_sweep_p(
    int64_t n_row, const int32_t* __restrict__ row_sim, const int32_t* __restrict__ simflag,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind, const double* __restrict__ val,
    const double* __restrict__ dinv, const double* __restrict__ b, const double* __restrict__ x_in,
    double* __restrict__ x_out, double omega, const int32_t* __restrict__ ptab, const double* __restrict__ pw,
    const double* __restrict__ xc, const uint8_t* __restrict__ cmask) {
  constexpr int VL = 8, NA = VL / LPR, NS = 4;
  const int lane = threadIdx.x % LPR, grp = threadIdx.x / LPR;
  const int64_t row = (int64_t)blockIdx.x * ROWS_PER_BLOCK + grp;
  if (row >= n_row) return;   // the row's LPR lanes leave together
  // rows in row order; rows of finished sims leave before their block loads (as k_mg_sweep)
  const int k0r = rowptr[row], k1 = rowptr[row + 1];
  if (simflag[2 * row_sim[row]] >= 0) return;   // the row's LPR lanes leave together
  double p0[NA], p1[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) p0[a] = p1[a] = 0.0;
  // batches of four steps, loaded before their sums (as mg_sweep_row)
  for (int kb = k0r + lane; kb < k1; kb += NS * VL) {
    int64_t cc[NS][NA];
    double bl[NS][NA][4], xv[NS][NA][2];
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const int k = min(kb + j * VL + a * LPR, k1 - 1);
        cc[j][a] = colind[k];
#pragma unroll
        for (int e = 0; e < 4; ++e) bl[j][a][e] = val[(int64_t)k * 4 + e];
      }
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int a = 0; a < NA; ++a) mg_prolonged(cc[j][a], ptab, pw, xc, cmask, x_in, xv[j][a][0], xv[j][a][1]);
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int a = 0; a < NA; ++a)
        if (kb + j * VL + a * LPR < k1) {
          p0[a] = p0[a] + dot2(bl[j][a][0], xv[j][a][0], bl[j][a][1], xv[j][a][1]);
          p1[a] = p1[a] + dot2(bl[j][a][2], xv[j][a][0], bl[j][a][3], xv[j][a][1]);
        }
  }
#pragma unroll
  for (int m = NA / 2; m > 0; m >>= 1)
#pragma unroll
    for (int a = 0; a < m; ++a) { p0[a] += p0[a + m]; p1[a] += p1[a + m]; }
  double a0 = p0[0], a1 = p1[0];
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) {
    a0 += __shfl_xor(a0, off, LPR);
    a1 += __shfl_xor(a1, off, LPR);
  }
  if (lane == 0) {
    const double r0 = b[row * 2] - a0, r1 = b[row * 2 + 1] - a1;
    const double* D = dinv + row * 4;
    double base0, base1;
    mg_prolonged(row, ptab, pw, xc, cmask, x_in, base0, base1);
    x_out[row * 2] = fma(omega, dot2(D[0], r0, D[1], r1), base0);
    x_out[row * 2 + 1] = fma(omega, dot2(D[2], r0, D[3], r1), base1);
  }
}

// b_c = R r_f on one coarse row per thread (R = transpose of the linear
// interpolation): fine node (2I + di, 2J + dj), di, dj in {-1, 0, 1}, weighs
// (1 or 1/2 per axis); the restriction table lists its row in (dj, di) order,
// -1 where it is off the grid or inactive.  Constrained coarse unknowns get 0.
// The nine row loads are issued together, then the products are added in
// table order.
__global__ void k_mg_restrict(int64_t n_crow, const int32_t* __restrict__ rtab, const double* __restrict__ rf,
                              const uint8_t* __restrict__ c_cmask, double* __restrict__ bc) {
  const int64_t R = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (R >= n_crow) return;
  int32_t fr[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) fr[q] = rtab[R * 9 + q];
  const uint8_t m0 = c_cmask[R * 2], m1 = c_cmask[R * 2 + 1];
  // every fine value is loaded at once (a -1 entry reads fine row 0, which
  // exists whenever this level has rows, and is not added)
  double v[9][2];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const double* src = rf + (int64_t)(fr[q] < 0 ? 0 : fr[q]) * 2;
    v[q][0] = src[0];
    v[q][1] = src[1];
  }
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    if (fr[q] < 0) continue;
    const double wy = q / 3 == 1 ? 1.0 : 0.5;
    const double wgt = wy * (q % 3 == 1 ? 1.0 : 0.5);
    a0 = fma(wgt, v[q][0], a0);
    a1 = fma(wgt, v[q][1], a1);
  }
  bc[R * 2] = m0 ? 0.0 : a0;
  bc[R * 2 + 1] = m1 ? 0.0 : a1;
}

// x_f += P x_c on one fine row per thread, from the prolongation table (the
// terms and order of mg_prolonged); constrained fine unknowns keep their
// value.
__global__ void k_mg_prolong(int64_t n_frow, const int32_t* __restrict__ ptab, const double* __restrict__ pw,
                             const double* __restrict__ xc, const uint8_t* __restrict__ f_cmask,
                             double* __restrict__ xf) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_frow) return;
  double x0, x1;
  mg_prolonged(r, ptab, pw, xc, f_cmask, xf, x0, x1);
  xf[r * 2] = x0;
  xf[r * 2 + 1] = x1;
}

// Coarsest level: dense matrix of each sim (n_s = 2 * rows, stride nmax),
// scattered from its BSR rows; one thread per BSR entry.
__global__ void k_mg_dense_fill(int64_t n_row, const int32_t* __restrict__ row_sim,
                                const int32_t* __restrict__ doff, const int32_t* __restrict__ rowptr,
                                const int32_t* __restrict__ colind, const double* __restrict__ val, int nmax,
                                double* __restrict__ dense) {
  const int64_t row = (int64_t)blockIdx.x * 2 + threadIdx.x / 32;   // 64 threads: two rows
  if (row >= n_row) return;
  const int k = rowptr[row] + (int)(threadIdx.x % 32);
  if (k >= rowptr[row + 1]) return;
  const int s = row_sim[row];
  const int r0 = doff[2 * s];
  double* A = dense + (int64_t)s * 2 * nmax * nmax;
  const int lr = (int)(row - r0), lc = colind[k] - r0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) A[(int64_t)(2 * lr + i) * nmax + 2 * lc + j] = val[(int64_t)k * 4 + i * 2 + j];
}

// In-place Gauss-Jordan inversion with partial pivoting in LDS, one
// workgroup per sim (n <= MG_DENSE_MAX).  dense[s] holds A (nmax x nmax,
// leading n x n used) followed by the inverse, stored transposed so that the
// per-V-cycle product reads it coalesced.  A zero pivot sets flag bit 16
// and leaves that column unreduced.
constexpr int GJ = 256;
__global__ void __launch_bounds__(GJ) k_mg_gauss_jordan(const int32_t* __restrict__ doff, int nmax,
                                                        double* __restrict__ dense, int32_t* __restrict__ flag) {
  const int s = blockIdx.x;
  const int n = 2 * doff[2 * s + 1];
  const double* Ag = dense + (int64_t)s * 2 * nmax * nmax;
  double* Vt = dense + (int64_t)s * 2 * nmax * nmax + (int64_t)nmax * nmax;
  __shared__ double A[MG_DENSE_MAX * MG_DENSE_MAX];
  __shared__ double F[MG_DENSE_MAX];
  __shared__ double sv[GJ];
  __shared__ int si[GJ];
  __shared__ int piv[MG_DENSE_MAX];
  __shared__ double pinv;
  for (int e = threadIdx.x; e < n * n; e += GJ) A[e] = Ag[(int64_t)(e / n) * nmax + e % n];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot: largest |A[i][k]|, i >= k; ties to the lowest row
    double best = -1.0;
    int bi = k;
    for (int i = k + threadIdx.x; i < n; i += GJ) {
      const double v = fabs(A[i * n + k]);
      if (v > best) { best = v; bi = i; }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = GJ / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        const double o = sv[threadIdx.x + w];
        const int oi = si[threadIdx.x + w];
        if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && oi < si[threadIdx.x])) {
          sv[threadIdx.x] = o;
          si[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    const int p = si[0];
    const bool singular = !(sv[0] > 0.0);
    __syncthreads();
    if (threadIdx.x == 0) piv[k] = singular ? k : p;
    if (singular) {
      if (threadIdx.x == 0) atomicOr(flag, 16);
      __syncthreads();
      continue;
    }
    if (p != k)
      for (int j = threadIdx.x; j < n; j += GJ) {
        const double t = A[k * n + j];
        A[k * n + j] = A[p * n + j];
        A[p * n + j] = t;
      }
    __syncthreads();
    if (threadIdx.x == 0) {
      pinv = 1.0 / A[k * n + k];
      A[k * n + k] = 1.0;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += GJ) A[k * n + j] *= pinv;
    for (int i = threadIdx.x; i < n; i += GJ) F[i] = (i == k) ? 0.0 : A[i * n + k];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += GJ)
      if (i != k) A[i * n + k] = 0.0;
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += GJ) {
      const int i = e / n, j = e % n;
      if (i != k) A[e] -= F[i] * A[k * n + j];
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = n - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k)
      for (int i = threadIdx.x; i < n; i += GJ) {
        const double t = A[i * n + k];
        A[i * n + k] = A[i * n + p];
        A[i * n + p] = t;
      }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n * n; e += GJ) {
    const int i = e / n, j = e % n;
    Vt[(int64_t)j * nmax + i] = A[e];
  }
}

// x = A^-1 b for sim s on the coarsest level: lane i (one wave, n <= 64)
// owns unknown i and reads the transposed inverse column by column.
__device__ __forceinline__ void mg_dense_lane(int s, int i, const int32_t* __restrict__ doff, int nmax,
                                              const double* __restrict__ dense, const double* __restrict__ b,
                                              double* __restrict__ x) {
  const int r0 = doff[2 * s], n = 2 * doff[2 * s + 1];
  if (i >= n) return;   // lanes past this sim's unknowns (nmax may be < 64) read nothing
  const double* Vt = dense + (int64_t)s * 2 * nmax * nmax + (int64_t)nmax * nmax;
  const double* bs = b + (int64_t)r0 * 2;
  double acc = 0.0;
  for (int j = 0; j < n; ++j) acc = fma(Vt[(int64_t)j * nmax + i], bs[j], acc);
  x[(int64_t)r0 * 2 + i] = acc;
}

__global__ void __launch_bounds__(64) k_mg_dense_apply(const int32_t* __restrict__ doff, int nmax,
                                                       const double* __restrict__ dense,
                                                       const double* __restrict__ b, double* __restrict__ x) {
  mg_dense_lane(blockIdx.x, threadIdx.x, doff, nmax, dense, b, x);
}

// Transfer tables of the fused tail, in the order the row functions above
// visit their terms.  rtab: per coarse row the 9 finer rows of the (dj, di)
// loop (-1 where the term is skipped).  ptab: per fine row the coarser rows
// of the (J, I) loop in order, -1 after the last; pw: their common weight.
__global__ void k_mg_rtab(int64_t n_crow, const int64_t* __restrict__ c_active, const int32_t* __restrict__ c_rowsim,
                          const SimDev* __restrict__ csims, const SimDev* __restrict__ fsims,
                          const int32_t* __restrict__ f_node_map, int32_t* __restrict__ tab) {
  const int64_t R = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (R >= n_crow) return;
  const int s = c_rowsim[R];
  const SimDev& C = csims[s];
  const SimDev& F = fsims[s];
  const int64_t loc = c_active[R] - C.node_base;
  const int I = (int)(loc % C.nna[0]) - 1, J = (int)(loc / C.nna[0]) - 1;
  int q = 0;
  for (int dj = -1; dj <= 1; ++dj)
    for (int di = -1; di <= 1; ++di, ++q) {
      const int j = 2 * J + dj, i = 2 * I + di;
      int32_t fr = -1;
      if (j >= -1 && j <= F.n[1] + 1 && i >= -1 && i <= F.n[0] + 1)
        fr = f_node_map[F.node_base + (i + 1) + (int64_t)F.nna[0] * (j + 1)];
      tab[R * 9 + q] = fr < 0 ? -1 : fr;
    }
}

__global__ void k_mg_ptab(int64_t n_frow, const int64_t* __restrict__ f_active, const int32_t* __restrict__ f_rowsim,
                          const SimDev* __restrict__ fsims, const SimDev* __restrict__ csims,
                          const int32_t* __restrict__ c_node_map, int32_t* __restrict__ tab, double* __restrict__ w) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_frow) return;
  const int s = f_rowsim[r];
  const SimDev& F = fsims[s];
  const SimDev& C = csims[s];
  const int64_t loc = f_active[r] - F.node_base;
  const int i = (int)(loc % F.nna[0]) - 1, j = (int)(loc / F.nna[0]) - 1;
  const int Ix0 = (i % 2 == 0) ? i / 2 : (i - 1) / 2, Ix1 = (i % 2 == 0) ? i / 2 : (i + 1) / 2;
  const int Jy0 = (j % 2 == 0) ? j / 2 : (j - 1) / 2, Jy1 = (j % 2 == 0) ? j / 2 : (j + 1) / 2;
  const double wx = Ix0 == Ix1 ? 1.0 : 0.5, wy = Jy0 == Jy1 ? 1.0 : 0.5;
  int q = 0;
  for (int J = Jy0; J <= Jy1; ++J) {
    if (J < -1 || J > C.n[1] + 1) continue;
    for (int I = Ix0; I <= Ix1; ++I) {
      if (I < -1 || I > C.n[0] + 1) continue;
      const int32_t cr = c_node_map[C.node_base + (I + 1) + (int64_t)C.nna[0] * (J + 1)];
      if (cr >= 0) tab[r * 4 + q++] = cr;
    }
  }
  for (; q < 4; ++q) tab[r * 4 + q] = -1;
  w[r] = wx * wy;
}

// The coarse tail of the V-cycle in one launch: one workgroup per sim runs
// the levels from the first one with at most MG_TAIL_ROWS rows per sim down
// to the dense solve and back, with the arithmetic of the level-by-level
// launches (same terms in the same order), a workgroup barrier standing in
// for each launch boundary.  Coarse levels are bound by launch and memory
// latency, so the tail keeps its working set close: the vectors of every
// tail level live in LDS, and each 4-lane group holds its row's blocks and
// inverted diagonal in registers across the sweeps of a level visit.
constexpr int MG_TAIL_THREADS = 1024;
constexpr int MG_TAIL_LPR = 4;                          // 256 row groups: one row each
constexpr int MG_TAIL_KB = (25 + MG_TAIL_LPR - 1) / MG_TAIL_LPR;   // blocks per lane (rows have <= 25)
constexpr int MG_TAIL_LDS_MAX = 64 * 1024;

struct TailRow {
  int col[MG_TAIL_KB];          // local column (row within the sim), -1 past the row end
  double v[MG_TAIL_KB][4];
  double D[4];
};

__device__ __forceinline__ void tail_load_row(const MgTailLevel& L, int row, int lane, TailRow& R, int r0) {
  const int k0 = L.rowptr[row], k1 = L.rowptr[row + 1];
  // every load is issued unconditionally (slots past the row end read its
  // first block and are then marked empty), so they are all in flight at once
  int ci[MG_TAIL_KB];
  double vv[MG_TAIL_KB][4];
#pragma unroll
  for (int j = 0; j < MG_TAIL_KB; ++j) {
    const int k = k0 + lane + MG_TAIL_LPR * j;
    const int kc = k < k1 ? k : k0;   // a row holds at least its diagonal block
    ci[j] = L.colind[kc];
#pragma unroll
    for (int e = 0; e < 4; ++e) vv[j][e] = L.val[(int64_t)kc * 4 + e];
  }
#pragma unroll
  for (int j = 0; j < MG_TAIL_KB; ++j) {
    const bool ok = k0 + lane + MG_TAIL_LPR * j < k1;
    R.col[j] = ok ? ci[j] - r0 : -1;
#pragma unroll
    for (int e = 0; e < 4; ++e) R.v[j][e] = ok ? vv[j][e] : 0.0;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) R.D[e] = L.dinv[(int64_t)row * 4 + e];
}

// mg_sweep_row<4> on a cached row, vectors in LDS (local rows)
__device__ __forceinline__ void tail_sweep(const TailRow& R, int g, int lane, const double* b, const double* xin,
                                           double* xout, int mode) {
  double a0 = 0.0, a1 = 0.0;
  if (mode != 0) {
    double p0[2] = {0.0, 0.0}, p1[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < MG_TAIL_KB; ++j) {
      if (R.col[j] >= 0) {
        const double x0 = xin[R.col[j] * 2], x1 = xin[R.col[j] * 2 + 1];
        p0[j & 1] = p0[j & 1] + dot2(R.v[j][0], x0, R.v[j][1], x1);
        p1[j & 1] = p1[j & 1] + dot2(R.v[j][2], x0, R.v[j][3], x1);
      }
    }
    p0[0] += p0[1];
    p1[0] += p1[1];
    a0 = p0[0];
    a1 = p1[0];
#pragma unroll
    for (int off = MG_TAIL_LPR / 2; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off, MG_TAIL_LPR);
      a1 += __shfl_xor(a1, off, MG_TAIL_LPR);
    }
  }
  if (lane == 0) {
    const double r0 = b[g * 2] - a0, r1 = b[g * 2 + 1] - a1;
    if (mode == 2) {
      xout[g * 2] = r0;
      xout[g * 2 + 1] = r1;
    } else {
      const double base0 = mode == 1 ? xin[g * 2] : 0.0;
      const double base1 = mode == 1 ? xin[g * 2 + 1] : 0.0;
      xout[g * 2] = fma(MG_OMEGA, dot2(R.D[0], r0, R.D[1], r1), base0);
      xout[g * 2 + 1] = fma(MG_OMEGA, dot2(R.D[2], r0, R.D[3], r1), base1);
    }
  }
}

__global__ void __launch_bounds__(MG_TAIL_THREADS) k_mg_tail(const MgTailLevel* __restrict__ lv, int nlev,
                                                             const int32_t* __restrict__ simflag,
                                                             const int32_t* __restrict__ doff, int nmax,
                                                             const double* __restrict__ dense,
                                                             const double* __restrict__ b_top,
                                                             double* __restrict__ x_top) {
  extern __shared__ double lds[];
  const int s = blockIdx.x;
  if (simflag && simflag[2 * s] >= 0) return;   // whole workgroup: the sim's solve is finished
  const int tid = threadIdx.x, lane = tid % MG_TAIL_LPR, g = tid / MG_TAIL_LPR;
  auto first_row = [&](const MgTailLevel& L) { return (int)L.sims[s].row_base; };
  auto end_row = [&](const MgTailLevel& L) { return s + 1 < L.nsim ? (int)L.sims[s + 1].row_base : L.n_row; };
  auto vec = [&](const MgTailLevel& L, int q) { return lds + L.lds + q * L.ldn; };   // q: 0 y, 1 r, 2 x, 3 b
  const bool odd = (MG_NU1 - 1 + MG_NU2) % 2 == 1;
  const bool pre_in_out = odd == ((MG_NU1 - 1) % 2 == 1);   // where the pre-smoothing iterate ends
  TailRow R;
  {
    const MgTailLevel& L = lv[0];
    const int r0 = first_row(L), n = end_row(L) - r0;
    double* b = vec(L, 3);
    for (int t = tid; t < 2 * n; t += MG_TAIL_THREADS) b[t] = b_top[(int64_t)r0 * 2 + t];
    __syncthreads();
  }
  // down: pre-smoothing, residual, restriction
  for (int m = 0; m < nlev; ++m) {
    const MgTailLevel& L = lv[m];
    const MgTailLevel& Cl = lv[m + 1];
    const int r0 = first_row(L), n = end_row(L) - r0;
    const bool mine = g < n;
    if (mine) tail_load_row(L, r0 + g, lane, R, r0);
    double *y = vec(L, 0), *r = vec(L, 1), *out = vec(L, 2), *b = vec(L, 3);
    double* xa = odd ? y : out;
    double* xb = odd ? out : y;
    if (mine) tail_sweep(R, g, lane, b, nullptr, xa, 0);
    __syncthreads();
    for (int k = 1; k < MG_NU1; ++k) {
      if (mine) tail_sweep(R, g, lane, b, xa, xb, 1);
      __syncthreads();
      double* t = xa; xa = xb; xb = t;
    }
    if (mine) tail_sweep(R, g, lane, b, xa, r, 2);
    __syncthreads();
    const int c0 = first_row(Cl), nc = end_row(Cl) - c0;
    double* bc = vec(Cl, 3);
    for (int t = tid; t < nc; t += MG_TAIL_THREADS) {
      const int32_t* tab = Cl.rtab + (int64_t)(c0 + t) * 9;
      int32_t fr[9];   // the table and mask loads are issued together
#pragma unroll
      for (int q = 0; q < 9; ++q) fr[q] = tab[q];
      const uint8_t m0 = Cl.cmask[(int64_t)(c0 + t) * 2], m1 = Cl.cmask[(int64_t)(c0 + t) * 2 + 1];
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        if (fr[q] < 0) continue;
        const double wy = q / 3 == 1 ? 1.0 : 0.5;
        const double wgt = wy * (q % 3 == 1 ? 1.0 : 0.5);
        a0 = fma(wgt, r[(fr[q] - r0) * 2], a0);
        a1 = fma(wgt, r[(fr[q] - r0) * 2 + 1], a1);
      }
      bc[t * 2] = m0 ? 0.0 : a0;
      bc[t * 2 + 1] = m1 ? 0.0 : a1;
    }
    __syncthreads();
  }
  // coarsest: dense solve (mg_dense_lane on the LDS vectors)
  {
    const MgTailLevel& C = lv[nlev];
    const int n = 2 * doff[2 * s + 1];
    const double* Vt = dense + (int64_t)s * 2 * nmax * nmax + (int64_t)nmax * nmax;
    const double* bs = vec(C, 3);
    if (tid < n) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc = fma(Vt[(int64_t)j * nmax + tid], bs[j], acc);
      vec(C, 2)[tid] = acc;
    }
    __syncthreads();
  }
  // up: prolongation, post-smoothing
  for (int m = nlev - 1; m >= 0; --m) {
    const MgTailLevel& L = lv[m];
    const MgTailLevel& Cl = lv[m + 1];
    const int r0 = first_row(L), n = end_row(L) - r0;
    const int c0 = first_row(Cl);
    const bool mine = g < n;
    if (mine) tail_load_row(L, r0 + g, lane, R, r0);
    double *y = vec(L, 0), *out = vec(L, 2), *b = vec(L, 3);
    const double* xc = vec(Cl, 2);
    double* xa = pre_in_out ? out : y;
    double* xb = pre_in_out ? y : out;
    for (int t = tid; t < n; t += MG_TAIL_THREADS) {
      const int32_t* tab = L.ptab + (int64_t)(r0 + t) * 4;
      int32_t cr[4];   // coarse rows first, then -1; all loads issued together
#pragma unroll
      for (int q = 0; q < 4; ++q) cr[q] = tab[q];
      const double w = L.pw[r0 + t];
      const uint8_t m0 = L.cmask[(int64_t)(r0 + t) * 2], m1 = L.cmask[(int64_t)(r0 + t) * 2 + 1];
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (cr[q] >= 0) {
          a0 = fma(w, xc[(cr[q] - c0) * 2], a0);
          a1 = fma(w, xc[(cr[q] - c0) * 2 + 1], a1);
        }
      if (!m0) xa[t * 2] += a0;
      if (!m1) xa[t * 2 + 1] += a1;
    }
    __syncthreads();
    for (int k = 0; k < MG_NU2; ++k) {
      if (mine) tail_sweep(R, g, lane, b, xa, xb, 1);
      __syncthreads();
      double* t = xa; xa = xb; xb = t;
    }
  }
  {
    const MgTailLevel& L = lv[0];
    const int r0 = first_row(L), n = end_row(L) - r0;
    const double* x = vec(L, 2);
    for (int t = tid; t < 2 * n; t += MG_TAIL_THREADS) x_top[(int64_t)r0 * 2 + t] = x[t];
  }
}

// Coarse-level group blocks in chunks: coarse stencil groups hold 4^l times
// the particles of a fine one, so each chunk (at most MG_CHUNK particles of
// one group) is one wave that stages its records in LDS and sums its 81
// local 2x2 blocks; k_mg_grp_sum then adds a group's chunks in order.
constexpr int MG_CHUNK = 64;

__device__ __forceinline__ double sel3m(int i, double v0, double v1, double v2) {
  return i == 0 ? v0 : (i == 1 ? v1 : v2);
}

__global__ void __launch_bounds__(64) k_mg_grp_chunk(const int32_t* __restrict__ chunk,
                                                     const double* __restrict__ pdat, double* __restrict__ part) {
  const int64_t ch = blockIdx.x;
  const int p0 = chunk[2 * ch], n = chunk[2 * ch + 1];
  __shared__ double rec[MG_CHUNK][28];
  for (int e = threadIdx.x; e < n * 28; e += 64) rec[e / 28][e % 28] = pdat[(int64_t)(p0 + e / 28) * PD2 + e % 28];
  __syncthreads();
  const int lane = threadIdx.x;
  const int j0 = lane, j1 = lane + 64 < 81 ? lane + 64 : 80;
  double K0[4] = {0.0, 0.0, 0.0, 0.0}, K1[4] = {0.0, 0.0, 0.0, 0.0};
  for (int q = 0; q < n; ++q) {
    const double* R = rec[q];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = h ? j1 : j0, a = j / 9, b = j % 9;
      const int ax = a % 3, ay = a / 3, bx = b % 3, by = b / 3;
      // R: T 0..15, wx 16..18, dwx 19..21, wy 22..24, dwy 25..27
      const double ga0 = sel3m(ax, R[19], R[20], R[21]) * sel3m(ay, R[22], R[23], R[24]);
      const double ga1 = sel3m(ax, R[16], R[17], R[18]) * sel3m(ay, R[25], R[26], R[27]);
      const double gb0 = sel3m(bx, R[19], R[20], R[21]) * sel3m(by, R[22], R[23], R[24]);
      const double gb1 = sel3m(bx, R[16], R[17], R[18]) * sel3m(by, R[25], R[26], R[27]);
      double* K = h ? K1 : K0;
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          K[r * 2 + c] += ga0 * (R[(2 * r) * 4 + 2 * c] * gb0 + R[(2 * r) * 4 + 2 * c + 1] * gb1) +
                          ga1 * (R[(2 * r + 1) * 4 + 2 * c] * gb0 + R[(2 * r + 1) * 4 + 2 * c + 1] * gb1);
    }
  }
  double* P = part + ch * GB2;
#pragma unroll
  for (int e = 0; e < 4; ++e) P[j0 * 4 + e] = K0[e];
  if (lane + 64 < 81)
#pragma unroll
    for (int e = 0; e < 4; ++e) P[j1 * 4 + e] = K1[e];
}

// gbuf[key] = sum of the key's chunks in chunk order (one wave per key).
__global__ void __launch_bounds__(256) k_mg_grp_sum(int64_t n_okeys, const int32_t* __restrict__ key_chunk,
                                                   const double* __restrict__ part, double* __restrict__ gbuf) {
  const int64_t key = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (key >= n_okeys) return;
  const int c0 = key_chunk[key], c1 = key_chunk[key + 1];
  if (c0 == c1) return;   // empty origin: never read
  for (int e = threadIdx.x % 64; e < GB2; e += 64) {
    double acc = 0.0;
    for (int ch = c0; ch < c1; ++ch) acc += part[(int64_t)ch * GB2 + e];
    gbuf[key * GB2 + e] = acc;
  }
}

// The same sums for levels whose groups hold many chunks: one workgroup per
// key, wave w adds chunks c0 + w, c0 + w + 16, ... in order, and the 16
// stripe sums meet in a fixed tree.
constexpr int MG_SUM_STRIPES = 16;
__global__ void __launch_bounds__(64 * MG_SUM_STRIPES) k_mg_grp_sum_wide(const int32_t* __restrict__ key_chunk,
                                                                         const double* __restrict__ part,
                                                                         double* __restrict__ gbuf) {
  const int64_t key = blockIdx.x;
  const int c0 = key_chunk[key], c1 = key_chunk[key + 1];
  if (c0 == c1) return;   // empty origin: never read (uniform over the workgroup)
  __shared__ double st[MG_SUM_STRIPES][GB2];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int e = lane; e < GB2; e += 64) {
    double acc = 0.0;
    for (int ch = c0 + w; ch < c1; ch += MG_SUM_STRIPES) acc += part[(int64_t)ch * GB2 + e];
    st[w][e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < GB2; e += 64 * MG_SUM_STRIPES) {
    double t[MG_SUM_STRIPES];
#pragma unroll
    for (int q = 0; q < MG_SUM_STRIPES; ++q) t[q] = st[q][e];
#pragma unroll
    for (int m = MG_SUM_STRIPES / 2; m > 0; m >>= 1)
#pragma unroll
      for (int q = 0; q < m; ++q) t[q] += t[q + m];
    gbuf[key * GB2 + e] = t[0];
  }
}

}  // namespace mpm

using namespace mpm;

static unsigned nb256(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

void mg_level_release(MgLevel* L) {
  if (L->sub) { ctx_release(L->sub); delete L->sub; }
  L->mask.release(); L->pmap.release(); L->vec.release(); L->chunk.release(); L->key_chunk.release();
  L->part.release(); L->pg.release(); L->nek.release(); L->pxs.release(); L->prec.release(); L->qsim.release();
  L->prgrp.release();
  delete L;
}

void mg_release(mpm_ctx* c) {
  for (MgLevel* L : c->mgl) mg_level_release(L);
  c->mgl.clear();
  c->mg_zero.release(); c->mg_inv.release(); c->mg_fine.release(); c->mg_dense.release(); c->mg_doff.release();
  c->mg_sims.release(); c->mg_tail.release(); c->mg_tab.release(); c->mg_tabw.release(); c->mg3_part.release();
  c->mg3_depth.release(); c->mg3_lam.release(); c->mg3_inv.release(); c->mg3_coef.release();
  c->mg_tail_first = -1;
  mg_drop_graphs(c);
  if (c->cap_stream) { (void)hipStreamDestroy(c->cap_stream); c->cap_stream = nullptr; }
  c->mg_ready = false;
}

// Chunks of the level's stencil groups, from its group starts (host side).
static int build_chunks(mpm_ctx* c, MgLevel* L) {
  mpm_ctx* sub = L->sub;
  std::vector<int32_t> gs(sub->n_okeys + 1);
  HIPC(c, hipMemcpyAsync(gs.data(), sub->gstart.p, gs.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  std::vector<int32_t> ch, kc(sub->n_okeys + 1);
  for (int64_t k = 0; k < sub->n_okeys; ++k) {
    kc[k] = (int32_t)(ch.size() / 2);
    for (int32_t p = gs[k]; p < gs[k + 1]; p += MG_CHUNK) {
      ch.push_back(p);
      ch.push_back(std::min(MG_CHUNK, gs[k + 1] - p));
    }
  }
  kc[sub->n_okeys] = (int32_t)(ch.size() / 2);
  L->n_chunks = (int64_t)(ch.size() / 2);
  L->max_key_chunks = 0;
  for (int64_t k = 0; k < sub->n_okeys; ++k) L->max_key_chunks = std::max(L->max_key_chunks, kc[k + 1] - kc[k]);
  if (L->chunk.ensure(std::max<size_t>(2, ch.size())) != hipSuccess ||
      L->key_chunk.ensure(kc.size()) != hipSuccess ||
      L->part.ensure((size_t)std::max<int64_t>(1, L->n_chunks) * GB2) != hipSuccess ||
      sub->gbuf.ensure((size_t)std::max<int64_t>(1, sub->n_okeys) * GB2) != hipSuccess)
    return c->fail(MPM_E_NOMEM, "multigrid chunk allocation failed");
  if (!ch.empty())
    HIPC(c, hipMemcpyAsync(L->chunk.p, ch.data(), ch.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(L->key_chunk.p, kc.data(), kc.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  return MPM_OK;
}

// Build (or re-prepare) the levels for the current prepare of c; pb is the
// fine problem.  Level contexts and their buffers are kept between prepares.
int mg_build(mpm_ctx* c, const mpm_problem* pb) {
  if (c->dim == 3 || c->up) return mg3_build(c, pb);
  if (c->dim != 2 || c->up) return c->fail(MPM_E_INVALID, "the multigrid preconditioner covers single-phase problems");
  const int nsim = c->nsim;
  const int64_t np = c->np;
  if (c->mg_inv.ensure(std::max<int64_t>(1, np)) != hipSuccess ||
      c->mg_fine.ensure(std::max<int64_t>(1, 2 * c->n_row * 2)) != hipSuccess ||
      c->mg_sims.ensure(nsim) != hipSuccess)
    return c->fail(MPM_E_NOMEM, "multigrid allocation failed");
  if (np) {
    k_mg_inv_perm<<<nb256(np), 256, 0, c->stream>>>(np, c->perm.p, c->mg_inv.p);
    LAUNCH_CHECK(c, "k_mg_inv_perm");
  }
  std::vector<mpm_grid> grids(pb->grids, pb->grids + nsim);
  const mpm_ctx* finer = c;
  const uint8_t* fmask = pb->bc_mask;
  size_t nl = 0;
  for (int l = 1; l <= MG_MAX_LEVELS; ++l) {
    // stop once the finer level is small enough for the dense solve
    int64_t worst = 0;
    bool shrinkable = false;
    for (int s = 0; s < nsim; ++s) {
      worst = std::max<int64_t>(worst, 2 * (finer->sim_row_start[s + 1] - finer->sim_row_start[s]));
      shrinkable = shrinkable || grids[s].ncell[0] > 1 || grids[s].ncell[1] > 1;
    }
    if (worst <= MG_DENSE_MAX || !shrinkable) break;
    for (int s = 0; s < nsim; ++s) {
      grids[s].h *= 2.0;
      grids[s].ncell[0] = std::max(1, (grids[s].ncell[0] + 1) / 2);
      grids[s].ncell[1] = std::max(1, (grids[s].ncell[1] + 1) / 2);
    }
    if (c->mgl.size() < (size_t)l) {
      MgLevel* L = new (std::nothrow) MgLevel();
      if (!L) return c->fail(MPM_E_NOMEM, "multigrid level allocation failed");
      c->mgl.push_back(L);
      L->sub = new (std::nothrow) mpm_ctx();
      if (!L->sub) return c->fail(MPM_E_NOMEM, "multigrid level allocation failed");
    }
    MgLevel* L = c->mgl[l - 1];
    mpm_ctx* sub = L->sub;
    sub->device = c->device;
    sub->stream = c->stream;
    sub->mg_level = true;
    L->grids = grids;
    // child descriptors (node bases as the child's prepare lays them out) for its mask
    std::vector<SimDev> cs(nsim);
    int64_t n_cnodes = 0;
    for (int s = 0; s < nsim; ++s) {
      SimDev& S = cs[s];
      S = SimDev{};
      for (int k = 0; k < 2; ++k) {
        S.n[k] = grids[s].ncell[k];
        S.nna[k] = grids[s].ncell[k] + 3;
        S.noa[k] = grids[s].ncell[k] + 1;
      }
      S.n[2] = 0; S.nna[2] = 1; S.noa[2] = 1;
      S.node_base = n_cnodes;
      n_cnodes += (int64_t)S.nna[0] * S.nna[1];
    }
    if (L->mask.ensure(std::max<int64_t>(1, 2 * n_cnodes)) != hipSuccess ||
        c->mg_zero.ensure(std::max<size_t>(c->mg_zero.n, (size_t)std::max<int64_t>(1, 2 * n_cnodes))) != hipSuccess)
      return c->fail(MPM_E_NOMEM, "multigrid mask allocation failed");
    HIPC(c, hipMemsetAsync(c->mg_zero.p, 0, c->mg_zero.n * sizeof(double), c->stream));
    HIPC(c, hipMemcpyAsync(c->mg_sims.p, cs.data(), nsim * sizeof(SimDev), hipMemcpyHostToDevice, c->stream));
    k_mg_mask<<<nb256(n_cnodes), 256, 0, c->stream>>>(n_cnodes, nsim, c->mg_sims.p, finer->sims.p, fmask,
                                                      L->mask.p);
    LAUNCH_CHECK(c, "k_mg_mask");
    mpm_problem cp = *pb;
    cp.mat.shape = 0;   // coarse levels are rediscretized with quadratic B-splines (a preconditioner only)
    cp.grids = L->grids.data();
    cp.bc_mask = L->mask.p;
    cp.bc_value = c->mg_zero.p;
    cp.react_mask = nullptr;
    int rc = mpm_prepare_impl(sub, &cp, nullptr, nullptr, nullptr);
    if (rc) return c->fail(rc, "multigrid level " + std::to_string(l) + ": " + sub->err);
    if (L->pmap.ensure(std::max<int64_t>(1, np)) != hipSuccess ||
        L->vec.ensure(std::max<int64_t>(1, 4 * sub->n_row * 2)) != hipSuccess ||
        sub->val.ensure(std::max<int64_t>(1, sub->nnzb * 4)) != hipSuccess ||
        sub->pdat.ensure(std::max<int64_t>(1, np) * PD2) != hipSuccess)
      return c->fail(MPM_E_NOMEM, "multigrid level allocation failed");
    if (np) {
      k_mg_pmap<<<nb256(np), 256, 0, c->stream>>>(np, sub->perm.p, c->mg_inv.p, L->pmap.p);
      LAUNCH_CHECK(c, "k_mg_pmap");
    }
    GUARD(build_chunks(c, L));
    finer = sub;
    fmask = L->mask.p;
    nl = l;
  }
  while (c->mgl.size() > nl) { mg_level_release(c->mgl.back()); c->mgl.pop_back(); }
  // fused coarse tail: from the first level whose sims all have at most
  // MG_TAIL_ROWS rows, when at least one smoothed level lies above the dense solve
  c->mg_tail_first = -1;
  for (size_t l = 0; l < nl && c->mg_tail_first < 0; ++l) {
    const mpm_ctx* L = l == 0 ? c : c->mgl[l - 1]->sub;
    int64_t mx = 0;
    for (int s = 0; s < nsim; ++s) mx = std::max<int64_t>(mx, L->sim_row_start[s + 1] - L->sim_row_start[s]);
    if (mx <= MG_TAIL_ROWS) c->mg_tail_first = (int)l;
  }
  // transfer tables of every level (restriction on the coarse side,
  // prolongation on the fine side): per level rtab, ptab, pw offsets
  {
    std::vector<int64_t> toff(3 * (nl + 1), -1);
    int64_t ntab = 0, nw = 0;
    for (size_t l = 0; l <= nl; ++l) {
      const mpm_ctx* L = l == 0 ? c : c->mgl[l - 1]->sub;
      if (l >= 1) { toff[3 * l] = ntab; ntab += L->n_row * 9; }
      if (l < nl) { toff[3 * l + 1] = ntab; ntab += L->n_row * 4; toff[3 * l + 2] = nw; nw += L->n_row; }
    }
    if (c->mg_tab.ensure(std::max<int64_t>(1, ntab)) != hipSuccess || c->mg_tabw.ensure(std::max<int64_t>(1, nw)) != hipSuccess)
      return c->fail(MPM_E_NOMEM, "multigrid table allocation failed");
    for (size_t l = 0; l <= nl; ++l) {
      const mpm_ctx* L = l == 0 ? c : c->mgl[l - 1]->sub;
      if (l >= 1 && L->n_row) {
        const mpm_ctx* Fn = l - 1 == 0 ? c : c->mgl[l - 2]->sub;
        k_mg_rtab<<<nb256(L->n_row), 256, 0, c->stream>>>(L->n_row, L->active_nodes.p, L->row_sim.p, L->sims.p,
                                                         Fn->sims.p, Fn->node_map.p, c->mg_tab.p + toff[3 * l]);
        LAUNCH_CHECK(c, "k_mg_rtab");
      }
      if (l < nl && L->n_row) {
        const mpm_ctx* Cn = c->mgl[l]->sub;
        k_mg_ptab<<<nb256(L->n_row), 256, 0, c->stream>>>(L->n_row, L->active_nodes.p, L->row_sim.p, L->sims.p,
                                                         Cn->sims.p, Cn->node_map.p, c->mg_tab.p + toff[3 * l + 1],
                                                         c->mg_tabw.p + toff[3 * l + 2]);
        LAUNCH_CHECK(c, "k_mg_ptab");
      }
    }
    c->mg_lvl_off = toff;
  }
  if (c->mg_tail_first >= 0) {
    // LDS layout of the tail: four vectors per level, sized for the largest sim
    const size_t first = (size_t)c->mg_tail_first;
    std::vector<int64_t> off;
    int64_t lds = 0;
    for (size_t l = first; l <= nl; ++l) {
      const mpm_ctx* L = l == 0 ? c : c->mgl[l - 1]->sub;
      int64_t mx = 0;
      for (int s = 0; s < nsim; ++s) mx = std::max<int64_t>(mx, L->sim_row_start[s + 1] - L->sim_row_start[s]);
      off.push_back(lds);
      off.push_back(2 * mx);
      lds += 4 * 2 * mx;
      off.push_back(l > first ? c->mg_lvl_off[3 * l] : -1);   // rtab (coarse side, within the tail)
      off.push_back(c->mg_lvl_off[3 * l + 1]);                 // ptab (fine side)
      off.push_back(c->mg_lvl_off[3 * l + 2]);                 // pw
    }
    if (lds * (int64_t)sizeof(double) > MG_TAIL_LDS_MAX) {
      c->mg_tail_first = -1;   // too large for one workgroup's LDS: level-by-level launches
    } else {
      c->mg_tab_off = off;
      c->mg_tail_lds = (int)(lds * sizeof(double));
      if (c->mg_tail.ensure(nl - first + 1) != hipSuccess)
        return c->fail(MPM_E_NOMEM, "multigrid tail allocation failed");
    }
  }
  // coarsest: dense per sim
  const mpm_ctx* C = nl ? c->mgl.back()->sub : c;
  std::vector<int32_t> doff(2 * nsim);
  int nmax = 1;
  for (int s = 0; s < nsim; ++s) {
    doff[2 * s] = (int32_t)C->sim_row_start[s];
    doff[2 * s + 1] = (int32_t)(C->sim_row_start[s + 1] - C->sim_row_start[s]);
    nmax = std::max(nmax, 2 * doff[2 * s + 1]);
  }
  if (nmax > MG_DENSE_MAX) return c->fail(MPM_E_INVALID, "multigrid coarsest level too large for the dense solve");
  c->mg_nmax = nmax;
  if (c->mg_doff.ensure(2 * nsim) != hipSuccess ||
      c->mg_dense.ensure((size_t)nsim * 2 * nmax * nmax) != hipSuccess)
    return c->fail(MPM_E_NOMEM, "multigrid dense allocation failed");
  HIPC(c, hipMemcpyAsync(c->mg_doff.p, doff.data(), doff.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  ++c->mg_gen;            // level buffers may have moved: captured V-cycles are stale
  mg_drop_graphs(c);
  c->mg_ready = true;
  return MPM_OK;
}

// Per Newton iteration, after the fine Jacobian (records in c->pdat) and its
// block-Jacobi inverse: level records, matrices, inverses, coarsest inverse.
int mg_setup(mpm_ctx* c) {
  if (c->dim == 3 || c->up) return mg3_setup(c);
  const int64_t np = c->np;
  for (MgLevel* L : c->mgl) {
    mpm_ctx* sub = L->sub;
    if (np) {
      k_mg_rec2<<<nb256(np), 256, 0, c->stream>>>(np, sub->xs.p, sub->psim.p, sub->sims.p, L->pmap.p, c->pdat.p,
                                                  sub->pdat.p);
      LAUNCH_CHECK(c, "k_mg_rec2");
    }
    if (L->n_chunks) {
      k_mg_grp_chunk<<<(unsigned)L->n_chunks, 64, 0, c->stream>>>(L->chunk.p, sub->pdat.p, L->part.p);
      LAUNCH_CHECK(c, "k_mg_grp_chunk");
    }
    if (sub->n_okeys && L->max_key_chunks >= MG_SUM_STRIPES) {
      k_mg_grp_sum_wide<<<(unsigned)sub->n_okeys, 64 * MG_SUM_STRIPES, 0, c->stream>>>(L->key_chunk.p, L->part.p,
                                                                                        sub->gbuf.p);
      LAUNCH_CHECK(c, "k_mg_grp_sum_wide");
    } else if (sub->n_okeys) {
      k_mg_grp_sum<<<(unsigned)((sub->n_okeys + 3) / 4), 256, 0, c->stream>>>(sub->n_okeys, L->key_chunk.p,
                                                                             L->part.p, sub->gbuf.p);
      LAUNCH_CHECK(c, "k_mg_grp_sum");
    }
    int rc = launch_jac2_blocks(sub, sub->val.p, true);
    if (!rc) rc = launch_bj_inv(sub, sub->val.p);
    if (rc) return c->fail(rc, "multigrid level setup: " + sub->err);
  }
  const mpm_ctx* C = c->mgl.empty() ? c : c->mgl.back()->sub;
  const double* Cval = c->mgl.empty() ? c->val.p : C->val.p;
  const int nmax = c->mg_nmax;
  HIPC(c, hipMemsetAsync(c->mg_dense.p, 0, (size_t)c->nsim * 2 * nmax * nmax * sizeof(double), c->stream));
  if (C->n_row) {
    k_mg_dense_fill<<<(unsigned)((C->n_row + 1) / 2), 64, 0, c->stream>>>(C->n_row, C->row_sim.p, c->mg_doff.p,
                                                                         C->rowptr.p, C->colind.p, Cval, nmax,
                                                                         c->mg_dense.p);
    LAUNCH_CHECK(c, "k_mg_dense_fill");
  }
  k_mg_gauss_jordan<<<(unsigned)c->nsim, GJ, 0, c->stream>>>(c->mg_doff.p, nmax, c->mg_dense.p, c->flag.p);
  LAUNCH_CHECK(c, "k_mg_gauss_jordan");
  if (c->mg_tail_first >= 0) {
    // device views of the tail levels (the operators' buffers are final here)
    const size_t nl = c->mgl.size();
    const size_t first = (size_t)c->mg_tail_first;
    c->mg_tail_h.clear();
    for (size_t l = first; l <= nl; ++l) {
      const mpm_ctx* L = l == 0 ? c : c->mgl[l - 1]->sub;
      const int64_t* o = &c->mg_tab_off[(l - first) * 5];
      MgTailLevel d;
      d.rowptr = L->rowptr.p;
      d.colind = L->colind.p;
      d.val = l == 0 ? c->val.p : L->val.p;
      d.dinv = l == 0 ? c->dinv.p : L->dinv.p;
      d.sims = L->sims.p;
      d.cmask = L->cmask.p;
      d.rtab = o[2] >= 0 ? c->mg_tab.p + o[2] : nullptr;
      d.ptab = o[3] >= 0 ? c->mg_tab.p + o[3] : nullptr;
      d.pw = o[4] >= 0 ? c->mg_tabw.p + o[4] : nullptr;
      d.n_row = (int32_t)L->n_row;
      d.nsim = c->nsim;
      d.lds = (int32_t)o[0];
      d.ldn = (int32_t)o[1];
      c->mg_tail_h.push_back(d);
    }
    HIPC(c, hipMemcpyAsync(c->mg_tail.p, c->mg_tail_h.data(), c->mg_tail_h.size() * sizeof(MgTailLevel),
                           hipMemcpyHostToDevice, c->stream));
  }
  return MPM_OK;
}

// Level view: its context, matrix and inverse diagonal.
namespace {
struct LevelView {
  const mpm_ctx* ctx;
  const double* val;
  const double* dinv;
};
}

static int sweep(mpm_ctx* c, const LevelView& L, const double* b, const double* xin, double* xout, int mode) {
  const int64_t n_row = L.ctx->n_row;
  if (!n_row) return MPM_OK;
  const unsigned g = (unsigned)((n_row + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK);
  const unsigned t = ROWS_PER_BLOCK * 8;
  const int32_t *rs = L.ctx->row_sim.p, *rp = L.ctx->rowptr.p, *ci = L.ctx->colind.p;
  switch (mode) {
    case 0: k_mg_sweep<8, 0><<<g, t, 0, c->lstream>>>(n_row, rs, c->simflag.p, rp, ci, L.val, L.dinv, b, xin, xout, MG_OMEGA); break;
    case 1: k_mg_sweep<8, 1><<<g, t, 0, c->lstream>>>(n_row, rs, c->simflag.p, rp, ci, L.val, L.dinv, b, xin, xout, MG_OMEGA); break;
    case 2: k_mg_sweep<8, 2><<<g, t, 0, c->lstream>>>(n_row, rs, c->simflag.p, rp, ci, L.val, L.dinv, b, xin, xout, MG_OMEGA); break;
    case 3: k_mg_sweep<8, 3><<<g, t, 0, c->lstream>>>(n_row, rs, c->simflag.p, rp, ci, L.val, L.dinv, b, xin, xout, MG_OMEGA); break;
    default: return c->fail(MPM_E_INVALID, "multigrid sweep mode");
  }
  LAUNCH_CHECK(c, "k_mg_sweep");
  return MPM_OK;
}

// x = M^-1 b on level l (vectors of that level); result written to out.
static int vcycle(mpm_ctx* c, size_t l, const double* b, double* out) {
  const size_t nl = c->mgl.size();
  if (c->mg_fuse && c->mg_tail_first >= 0 && l == (size_t)c->mg_tail_first) {
    k_mg_tail<<<(unsigned)c->nsim, MG_TAIL_THREADS, c->mg_tail_lds, c->lstream>>>(
        c->mg_tail.p, (int)(nl - l), c->simflag.p, c->mg_doff.p, c->mg_nmax, c->mg_dense.p, b, out);
    LAUNCH_CHECK(c, "k_mg_tail");
    return MPM_OK;
  }
  if (l == nl) {
    k_mg_dense_apply<<<(unsigned)c->nsim, 64, 0, c->lstream>>>(c->mg_doff.p, c->mg_nmax, c->mg_dense.p, b, out);
    LAUNCH_CHECK(c, "k_mg_dense_apply");
    return MPM_OK;
  }
  const mpm_ctx* ctx = l == 0 ? c : c->mgl[l - 1]->sub;
  const LevelView V{ctx, l == 0 ? c->val.p : ctx->val.p, l == 0 ? c->dinv.p : ctx->dinv.p};
  const int64_t nv = ctx->n_row * 2;
  double* y = l == 0 ? c->mg_fine.p : c->mgl[l - 1]->vec.p;            // sweep ping-pong partner
  double* r = l == 0 ? c->mg_fine.p + nv : c->mgl[l - 1]->vec.p + nv;  // residual
  // the sweeps alternate between out and y; start where the last one ends in out
  const bool odd = (MG_NU1 - 1 + MG_NU2) % 2 == 1;
  double* xa = odd ? y : out;
  double* xb = odd ? out : y;
  int k_first = 1;
  if (c->mg_fuse && MG_NU1 >= 2) {   // the first two sweeps in one pass
    GUARD(sweep(c, V, b, nullptr, xb, 3));
    std::swap(xa, xb);
    k_first = 2;
  } else {
    GUARD(sweep(c, V, b, nullptr, xa, 0));
  }
  for (int k = k_first; k < MG_NU1; ++k) { GUARD(sweep(c, V, b, xa, xb, 1)); std::swap(xa, xb); }
  GUARD(sweep(c, V, b, xa, r, 2));
  // coarse correction
  MgLevel* CL = c->mgl[l];
  const mpm_ctx* C = CL->sub;
  double* xc = CL->vec.p + 2 * C->n_row * 2;
  double* bc = CL->vec.p + 3 * C->n_row * 2;
  if (C->n_row) {
    k_mg_restrict<<<nb256(C->n_row), 256, 0, c->lstream>>>(C->n_row, c->mg_tab.p + c->mg_lvl_off[3 * (l + 1)], r,
                                                          C->cmask.p, bc);
    LAUNCH_CHECK(c, "k_mg_restrict");
  }
  GUARD(vcycle(c, l + 1, bc, xc));
  int k_post = 0;
  if (c->mg_fuse && MG_NU2 >= 1 && l >= 1) {   // prolongation folded into the first post-smoothing sweep
    // (coarse levels only: on the finest the per-neighbour table reads cost more than the launch)
    if (ctx->n_row) {
      k_mg_sweep_p<8><<<(unsigned)((ctx->n_row + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK), ROWS_PER_BLOCK * 8, 0,
                        c->lstream>>>(
          ctx->n_row, ctx->row_sim.p, c->simflag.p, ctx->rowptr.p, ctx->colind.p, V.val, V.dinv, b, xa, xb,
          MG_OMEGA, c->mg_tab.p + c->mg_lvl_off[3 * l + 1], c->mg_tabw.p + c->mg_lvl_off[3 * l + 2], xc,
          ctx->cmask.p);
      LAUNCH_CHECK(c, "k_mg_sweep_p");
    }
    std::swap(xa, xb);
    k_post = 1;
  } else if (ctx->n_row) {
    k_mg_prolong<<<nb256(ctx->n_row), 256, 0, c->lstream>>>(ctx->n_row, c->mg_tab.p + c->mg_lvl_off[3 * l + 1],
                                                           c->mg_tabw.p + c->mg_lvl_off[3 * l + 2], xc, ctx->cmask.p,
                                                           xa);
    LAUNCH_CHECK(c, "k_mg_prolong");
  }
  for (int k = k_post; k < MG_NU2; ++k) { GUARD(sweep(c, V, b, xa, xb, 1)); std::swap(xa, xb); }
  if (xa != out) return c->fail(MPM_E_INVALID, "multigrid sweep parity");   // excluded by the choice of xa above
  return MPM_OK;
}

static void drop_graph(mpm_ctx::MgGraph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g = mpm_ctx::MgGraph{};
}

void mg_drop_graphs(mpm_ctx* c) {
  drop_graph(c->mg_exec[0]);
  drop_graph(c->mg_exec[1]);
}

// x = M^-1 b.  The V-cycle's launch sequence is fixed for a hierarchy and a
// pair of vectors, so it is captured once into a HIP graph (on a private
// stream: the caller's may be the null stream) and replayed with a single
// launch; the kernels read the Krylov flags, the level matrices and (3x3
// blocks) the Chebyshev coefficients at run time.
int mg_vcycle(mpm_ctx* c, const double* b, double* x) {
  const bool blk3 = c->dim == 3 || c->up;
  c->lstream = c->stream;
  if (!c->mg_graph) return blk3 ? mg3_vcycle(c, b, x) : vcycle(c, 0, b, x);
  const void* key[5] = {b, x, c->val.p, c->dinv.p, blk3 ? (const void*)c->mg3_coef.p : (const void*)c->simflag.p};
  mpm_ctx::MgGraph* hit = nullptr;
  for (auto& g : c->mg_exec)
    if (g.exec && g.gen == c->mg_gen && std::equal(key, key + 5, g.key)) hit = &g;
  if (!hit) {
    // an empty or stale slot, else evict the two slots alternately
    mpm_ctx::MgGraph* slot = nullptr;
    for (auto& e : c->mg_exec)
      if (!slot && (!e.exec || e.gen != c->mg_gen)) slot = &e;
    if (!slot) slot = &c->mg_exec[c->mg_next ^= 1];
    mpm_ctx::MgGraph& g = *slot;
    drop_graph(g);
    if (!c->cap_stream) HIPC(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPC(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipStream_t saved = c->stream;
    c->lstream = c->stream = c->cap_stream;   // every launch of the cycle goes to the capture
    int rc = blk3 ? mg3_vcycle(c, b, x) : vcycle(c, 0, b, x);
    c->lstream = c->stream = saved;
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
    if (rc || ec != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (rc) return rc;
      return c->fail(MPM_E_HIP, std::string("V-cycle capture: ") + hipGetErrorString(ec));
    }
    ec = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ec != hipSuccess) { g.exec = nullptr; return c->fail(MPM_E_HIP, std::string("V-cycle graph: ") + hipGetErrorString(ec)); }
    std::copy(key, key + 5, g.key);
    g.gen = c->mg_gen;
    hit = &g;
  }
  HIPC(c, hipGraphLaunch(hit->exec, c->stream));
  return MPM_OK;
}
