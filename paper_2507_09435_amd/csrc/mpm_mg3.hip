// Geometric multigrid V-cycle for operators of 3x3 blocks -- 3-D single-phase
// problems and plane-strain u-p problems (two displacements and the pore
// pressure per node): the analogue of the algebraic multigrid the paper pairs
// with its iterative solver (Sec. 2.2, Remark 2), built on the background grid.
//
// Level l uses grids of 2^l h with ceil(n / 2^l) cells per axis and the same
// origin.  Its operator is rediscretized from the particles: the finest
// level's tangent records (V0 dP/dF at the current iterate) are contracted
// with the level's own B-spline gradients by the same assembly as the finest
// matrix (u-p: the 7x7 tables of V0 d(P, s1, vv)/d(dF, p, grad p), through
// the row gather).  Transfers are trilinear (plane strain: bilinear)
// interpolation of node values
// (prolongation) and its transpose (restriction).  A coarse node is
// constrained where the finer node at its position is, and nodes without
// material as on every level.  Smoothing: a Chebyshev polynomial of degree
// MG3_DEG in the block-Jacobi-scaled operator D^-1 A (3x3 blocks) over
// [MG3_LO, MG3_HI] x lambda_max before and after the coarse correction, with
// lambda_max estimated per level and simulation by power iteration whenever
// the operators change.  (Damped block-Jacobi, which suits the plane-strain levels, diverges
// here: lambda_max(D^-1 A) is about 6 for these 3-D operators, so w = 0.6
// amplifies the stiff modes.)  Each simulation's coarsest level is inverted
// densely (Gauss-Jordan with partial pivoting).
//
// Depth per simulation: a simulation's coarsest level is the first on which
// it has at most MG3_DENSE_MAX unknowns, as if it were solved alone; the
// hierarchy goes as deep as the largest simulation needs, and the levels
// below a simulation's own coarsest carry its rows without touching them
// (smoothing, residuals, transfers and the power iteration skip them).  A
// batch then preconditions every simulation as its single solve does.  This
// matters for the u-p operators: coarsened past the consolidation length
// sqrt(c_v dt) the rediscretized operator stops approximating the fine one,
// and a small simulation taken to a large one's depth no longer converges.
//
// Quadrature particles: a coarse level's stencil groups hold 2^(dim l) times
// the particles of a fine group, so the level is not assembled from every
// particle.  Each non-empty origin o of the level (the particles whose
// stencil starts at o, that is, inside the dual cell [o + 1/2, o + 3/2] H)
// is represented by NG = 2^dim quadrature particles at the 2-point Gauss
// points of that dual cell, each carrying 1/NG of the sum of its particles'
// tables (V0 included).  All of them share the origin o, so the level's
// pattern is unchanged; the coarse operator is a coarser quadrature of the
// same rediscretization (a preconditioner only), and its assembly costs
// about 1/2^dim of the finer level's.
#include <algorithm>
#include <cmath>

#include "mpm_internal.hpp"

namespace mpm {

constexpr int MG3_DEG = 3;                // Chebyshev degree of the pre- and post-smoothing
constexpr double MG3_LO = 0.05;           // lower end of the Chebyshev interval (fraction of lambda_max)
constexpr int MG3_POWER = 20;             // power iterations for lambda_max(D^-1 A)
// upper end of the Chebyshev interval over the power estimate: the u-p
// operators are close to normal and the estimate approaches lambda_max from
// below (0.84 - 0.96 of it after 20 steps on oracle matrices); the 3-D ones
// are not, and ||D^-1 A v|| already reaches it
constexpr double MG3_HI_3D = 1.1, MG3_HI_UP = 1.3;
constexpr int MG3_MAX_LEVELS = 12;
constexpr int MG3_DENSE_MAX = 384;        // coarsest unknowns per simulation (inverted in global memory)
constexpr int MG3_LPR = 8;                // lanes per row in the sweeps

// Rows of level lev that are smoothed (their simulation's coarsest level is deeper).
__device__ __forceinline__ bool mg3_smooths(const int32_t* __restrict__ row_sim, const int32_t* __restrict__ depth,
                                            int64_t row, int lev) {
  return depth[row_sim[row]] > lev;
}

__device__ __forceinline__ int sim_of_node3(const SimDev* sims, int nsim, int64_t node) {
  int s = 0;
  while (s + 1 < nsim && node >= sims[s + 1].node_base) ++s;
  return s;
}

__device__ __forceinline__ void node_ijk(const SimDev& S, int64_t node, int& i, int& j, int& k) {
  int64_t loc = node - S.node_base;
  i = (int)(loc % S.nna[0]) - 1;
  loc /= S.nna[0];
  j = (int)(loc % S.nna[1]) - 1;
  k = (int)(loc / S.nna[1]) - 1;
}

__device__ __forceinline__ int64_t node_id(const SimDev& S, int i, int j, int k) {
  return S.node_base + (i + 1) + (int64_t)S.nna[0] * ((j + 1) + (int64_t)S.nna[1] * (k + 1));
}

__global__ void k_mg_inv_perm3(int64_t np, const int32_t* __restrict__ perm, int32_t* __restrict__ inv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) inv[perm[i]] = (int32_t)i;
}

// Level particle i (the level's sorted order) -> the finest level's sorted index.
__global__ void k_mg_pmap3(int64_t np, const int32_t* __restrict__ perm, const int32_t* __restrict__ inv,
                           int32_t* __restrict__ pmap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) pmap[i] = inv[perm[i]];
}

constexpr int MG3_CHUNK = 64;   // particles per chunk of the group sums

// Chunk sums of the finest tables in a level's sorted order: chunk j covers
// particles [start, start + count) of one origin; entry f sums, in order,
// frec[pmap[p] * stride + f] for f < nent.
__global__ void __launch_bounds__(128) k_mg3_chunk_sum(int64_t n_chunks, const int32_t* __restrict__ chunk,
                                                       const int32_t* __restrict__ pmap,
                                                       const double* __restrict__ frec, int stride, int nent,
                                                       double* __restrict__ part) {
  const int64_t j = blockIdx.x;
  if (j >= n_chunks) return;
  const int f = threadIdx.x;
  if (f >= nent) return;
  const int32_t p0 = chunk[2 * j], n = chunk[2 * j + 1];
  double s = 0.0;
  int k = 0;
  for (; k + 4 <= n; k += 4) {   // four independent loads, then the sums in order
    const double a0 = frec[(int64_t)pmap[p0 + k] * stride + f];
    const double a1 = frec[(int64_t)pmap[p0 + k + 1] * stride + f];
    const double a2 = frec[(int64_t)pmap[p0 + k + 2] * stride + f];
    const double a3 = frec[(int64_t)pmap[p0 + k + 3] * stride + f];
    s += a0;
    s += a1;
    s += a2;
    s += a3;
  }
  for (; k < n; ++k) s += frec[(int64_t)pmap[p0 + k] * stride + f];
  part[j * nent + f] = s;
}

// Quadrature particle tables of non-empty origin j: the origin's chunk sums
// in order, times 1/ng, into each of its ng particles (entries f < nent).
__global__ void __launch_bounds__(128) k_mg3_qrec(int64_t n_nek, const int32_t* __restrict__ nek,
                                                  const int32_t* __restrict__ key_chunk,
                                                  const double* __restrict__ part, int nent,
                                                  const int32_t* __restrict__ pg, int ng, int stride,
                                                  double* __restrict__ prec) {
  const int64_t j = blockIdx.x;
  if (j >= n_nek) return;
  const int f = threadIdx.x;
  if (f >= nent) return;
  const int32_t key = nek[j];
  double s = 0.0;
  for (int32_t c = key_chunk[key]; c < key_chunk[key + 1]; ++c) s += part[(int64_t)c * nent + f];
  s *= 1.0 / ng;
  const int64_t q0 = pg[key];
  for (int g = 0; g < ng; ++g) prec[(q0 + g) * stride + f] = s;
}

// Plane-strain u-p quadrature particles: their level weights and derivatives
// (record entries 49 .. 60), fixed for the prepare.
__global__ void k_mgup_qweights(int64_t npp, const double* __restrict__ pxs, const int32_t* __restrict__ psim_q,
                                const SimDev* __restrict__ sims, double* __restrict__ prec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npp) return;
  Stencil<2> st;
  make_stencil<2>(sims[psim_q ? psim_q[i] : 0], pxs, npp, i, st);
  double* C = prec + i * PU2;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C[49 + a] = st.w[0][a];
    C[52 + a] = st.dw[0][a];
    C[55 + a] = st.w[1][a];
    C[58 + a] = st.dw[1][a];
  }
}

// 3-D quadrature particles: their level weights and derivatives per axis
// (record entries PT3 .. PTW3 - 1), fixed for the prepare.
__global__ void k_mg3_qweights(int64_t npp, const double* __restrict__ pxs, const int32_t* __restrict__ psim_q,
                               const SimDev* __restrict__ sims, double* __restrict__ prec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npp) return;
  Stencil<3> st;
  make_stencil<3>(sims[psim_q[i]], pxs, npp, i, st);
  double* C = prec + i * PTW3 + PT3;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C[6 * ax + a] = st.w[ax][a];
      C[6 * ax + 3 + a] = st.dw[ax][a];
    }
}

// Coarse full-grid mask from the next finer one (the fine node at the same
// position, clamped into the fine grid).
__global__ void k_mg3_mask(int64_t n_cnodes, int nsim, int dim, const SimDev* __restrict__ csims,
                           const SimDev* __restrict__ fsims, const uint8_t* __restrict__ fmask,
                           uint8_t* __restrict__ cmask) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_cnodes) return;
  const int s = sim_of_node3(csims, nsim, g);
  const SimDev& C = csims[s];
  const SimDev& F = fsims[s];
  int I, J, K;
  node_ijk(C, g, I, J, K);
  const int i = min(max(2 * I, -1), F.n[0] + 1), j = min(max(2 * J, -1), F.n[1] + 1),
            k = dim == 3 ? min(max(2 * K, -1), F.n[2] + 1) : K;   // plane strain: the one z layer
  const int64_t fn = node_id(F, i, j, k);
#pragma unroll
  for (int c = 0; c < 3; ++c) cmask[g * 3 + c] = fmask[fn * 3 + c];
}

// Row product of MG3_LPR lanes: y = (A x)_row (blocks k of a row summed in
// lane k mod MG3_LPR, then a fixed butterfly; every lane ends with the sum).
__device__ __forceinline__ void mg3_row_product(int64_t row, int lane, const int32_t* __restrict__ rowptr,
                                                const int32_t* __restrict__ colind, const double* __restrict__ val,
                                                const double* __restrict__ x, double& y0, double& y1, double& y2) {
  y0 = y1 = y2 = 0.0;
  const int32_t k1 = rowptr[row + 1];
  for (int32_t k = rowptr[row] + lane; k < k1; k += MG3_LPR) {
    const double* B = val + (int64_t)k * 9;
    const double* xc = x + (int64_t)colind[k] * 3;
    const double x0 = xc[0], x1 = xc[1], x2 = xc[2];
    y0 += B[0] * x0 + B[1] * x1 + B[2] * x2;
    y1 += B[3] * x0 + B[4] * x1 + B[5] * x2;
    y2 += B[6] * x0 + B[7] * x1 + B[8] * x2;
  }
#pragma unroll
  for (int off = MG3_LPR / 2; off > 0; off >>= 1) {
    y0 += __shfl_xor(y0, off, MG3_LPR);
    y1 += __shfl_xor(y1, off, MG3_LPR);
    y2 += __shfl_xor(y2, off, MG3_LPR);
  }
}

// One Chebyshev step per row: z = D^-1 (b - A x_in) (x_in null: x = 0),
// d = c0 d + c1 z, x_out = x_in + d, with (c0, c1) = coef[2 s .. 2 s + 1]
// of the row's simulation s.  d is updated in place (row-local).  Rows of
// simulations not smoothed on this level are left alone.
__global__ void __launch_bounds__(256) k_mg3_cheb(int64_t n_row, int lev, const int32_t* __restrict__ row_sim,
                                                  const int32_t* __restrict__ depth, const int32_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ colind, const double* __restrict__ val,
                                                  const double* __restrict__ dinv, const double* __restrict__ b,
                                                  const double* __restrict__ x_in, double* __restrict__ x_out,
                                                  double* __restrict__ d, const double* __restrict__ coef, bool first) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / MG3_LPR;
  const int lane = threadIdx.x % MG3_LPR;
  if (row >= n_row || !mg3_smooths(row_sim, depth, row, lev)) return;   // a row's lanes leave together
  double y0 = 0.0, y1 = 0.0, y2 = 0.0;
  if (x_in) mg3_row_product(row, lane, rowptr, colind, val, x_in, y0, y1, y2);
  if (lane != 0) return;
  const int s = row_sim[row];
  const double c0 = coef[2 * s], c1 = coef[2 * s + 1];
  const double r0 = b[row * 3] - y0, r1 = b[row * 3 + 1] - y1, r2 = b[row * 3 + 2] - y2;
  const double* D = dinv + row * 9;
  const double z[3] = {D[0] * r0 + D[1] * r1 + D[2] * r2, D[3] * r0 + D[4] * r1 + D[5] * r2,
                       D[6] * r0 + D[7] * r1 + D[8] * r2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double dn = (first ? 0.0 : c0 * d[row * 3 + c]) + c1 * z[c];
    d[row * 3 + c] = dn;
    x_out[row * 3 + c] = (x_in ? x_in[row * 3 + c] : 0.0) + dn;
  }
}

// r = b - A x on the smoothed rows.
__global__ void __launch_bounds__(256) k_mg3_resid(int64_t n_row, int lev, const int32_t* __restrict__ row_sim,
                                                   const int32_t* __restrict__ depth, const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ colind, const double* __restrict__ val,
                                                   const double* __restrict__ b, const double* __restrict__ x,
                                                   double* __restrict__ r) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / MG3_LPR;
  const int lane = threadIdx.x % MG3_LPR;
  if (row >= n_row || !mg3_smooths(row_sim, depth, row, lev)) return;
  double y0, y1, y2;
  mg3_row_product(row, lane, rowptr, colind, val, x, y0, y1, y2);
  if (lane != 0) return;
  r[row * 3] = b[row * 3] - y0;
  r[row * 3 + 1] = b[row * 3 + 1] - y1;
  r[row * 3 + 2] = b[row * 3 + 2] - y2;
}

// Power iteration for lambda_max(D^-1 A), per simulation: w = D^-1 A v on
// the smoothed rows (0 on the others), and per row w.w.
__global__ void __launch_bounds__(256) k_mg3_pow(int64_t n_row, int lev, const int32_t* __restrict__ row_sim,
                                                 const int32_t* __restrict__ depth, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ colind, const double* __restrict__ val,
                                                 const double* __restrict__ dinv, const double* __restrict__ v,
                                                 double* __restrict__ w, double* __restrict__ rowww) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / MG3_LPR;
  const int lane = threadIdx.x % MG3_LPR;
  if (row >= n_row) return;
  double z0 = 0.0, z1 = 0.0, z2 = 0.0;
  if (mg3_smooths(row_sim, depth, row, lev)) {
    double y0, y1, y2;
    mg3_row_product(row, lane, rowptr, colind, val, v, y0, y1, y2);
    const double* D = dinv + row * 9;
    z0 = D[0] * y0 + D[1] * y1 + D[2] * y2;
    z1 = D[3] * y0 + D[4] * y1 + D[5] * y2;
    z2 = D[6] * y0 + D[7] * y1 + D[8] * y2;
  }
  if (lane != 0) return;
  w[row * 3] = z0;
  w[row * 3 + 1] = z1;
  w[row * 3 + 2] = z2;
  rowww[row] = z0 * z0 + z1 * z1 + z2 * z2;
}

// One workgroup per simulation: ||w||^2 over its rows (fixed order), then
// lambda[s] = ||w|| and inv[s] = 1 / ||w|| (the next vector's scale).  A zero
// or non-finite norm keeps lambda[s] and zeroes the simulation's vector.
// first: lambda[s] starts at 1.
__global__ void __launch_bounds__(256) k_mg3_pow_sim(int64_t n_row, int nsim, const SimDev* __restrict__ sims,
                                                     const double* __restrict__ rowww, double* __restrict__ inv,
                                                     double* __restrict__ lambda, bool first) {
  __shared__ double sa[256];
  const int s = blockIdx.x;
  const int64_t r0 = sims[s].row_base, r1 = s + 1 < nsim ? sims[s + 1].row_base : n_row;
  double a = 0.0;
  for (int64_t k = r0 + threadIdx.x; k < r1; k += 256) a += rowww[k];
  sa[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sa[threadIdx.x] += sa[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ww = sa[0];
    if (first) lambda[s] = 1.0;
    if (ww > 0.0 && isfinite(ww)) {
      const double nw = sqrt(ww);
      lambda[s] = nw;
      inv[s] = 1.0 / nw;
    } else {
      inv[s] = 0.0;
    }
  }
}

// v = inv[s] w on the rows of simulation s; the first vector (w null): a
// fixed pseudo-random field hashed from the row's index within its
// simulation and the component, so a simulation starts from the same vector
// alone or in any batch.
__global__ void k_mg3_scale(int64_t n, const int32_t* __restrict__ row_sim, const SimDev* __restrict__ sims,
                            const double* __restrict__ w, const double* __restrict__ inv, double* __restrict__ v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int s = row_sim[e / 3];
  if (w) { v[e] = inv[s] * w[e]; return; }
  const uint64_t el = (uint64_t)(e - 3 * sims[s].row_base);
  uint64_t h = el * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  h ^= h >> 31; h *= 0xBF58476D1CE4E5B9ull; h ^= h >> 29;
  v[e] = (double)(h >> 11) * (1.0 / 9007199254740992.0) + 0.5;
}

// Restriction (transpose of trilinear interpolation) from level lev: coarse
// row (I, J, K) gathers the fine rows at 2I + {-1, 0, 1} per axis with
// weights 1/2, 1, 1/2; constrained coarse unknowns get 0.  Rows of
// simulations not smoothed on level lev are skipped.
__global__ void k_mg3_restrict(int64_t n_crow, int dim, int lev, const int32_t* __restrict__ depth,
                               const int64_t* __restrict__ c_active,
                               const int32_t* __restrict__ c_rowsim, const SimDev* __restrict__ csims,
                               const SimDev* __restrict__ fsims, const int32_t* __restrict__ f_node_map,
                               const double* __restrict__ rf, const uint8_t* __restrict__ c_cmask,
                               double* __restrict__ bc) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n_crow || !mg3_smooths(c_rowsim, depth, row, lev)) return;
  const int s = c_rowsim[row];
  const SimDev& C = csims[s];
  const SimDev& F = fsims[s];
  int I, J, K;
  node_ijk(C, c_active[row], I, J, K);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  const int dk0 = dim == 3 ? -1 : 0, dk1 = dim == 3 ? 1 : 0;   // plane strain: the one z layer
  for (int dk = dk0; dk <= dk1; ++dk) {
    const int k = dim == 3 ? 2 * K + dk : K;
    if (k < -1 || k > F.n[2] + 1) continue;
    for (int dj = -1; dj <= 1; ++dj) {
      const int j = 2 * J + dj;
      if (j < -1 || j > F.n[1] + 1) continue;
      for (int di = -1; di <= 1; ++di) {
        const int i = 2 * I + di;
        if (i < -1 || i > F.n[0] + 1) continue;
        const int32_t fr = f_node_map[node_id(F, i, j, k)];
        if (fr < 0) continue;
        const double w = (di ? 0.5 : 1.0) * (dj ? 0.5 : 1.0) * (dk ? 0.5 : 1.0);
        a0 += w * rf[(int64_t)fr * 3];
        a1 += w * rf[(int64_t)fr * 3 + 1];
        a2 += w * rf[(int64_t)fr * 3 + 2];
      }
    }
  }
  bc[row * 3] = c_cmask[row * 3] ? 0.0 : a0;
  bc[row * 3 + 1] = c_cmask[row * 3 + 1] ? 0.0 : a1;
  bc[row * 3 + 2] = c_cmask[row * 3 + 2] ? 0.0 : a2;
}

// Prolongation added to x on level lev: fine node (i, j, k) takes, per
// axis, coarse node i/2 (i even) or the mean of (i-1)/2 and (i+1)/2 (i odd);
// constrained fine unknowns, and rows not smoothed on lev, are left alone.
__global__ void k_mg3_prolong_add(int64_t n_frow, int dim, int lev, const int32_t* __restrict__ depth,
                                  const int64_t* __restrict__ f_active,
                                  const int32_t* __restrict__ f_rowsim, const SimDev* __restrict__ fsims,
                                  const SimDev* __restrict__ csims, const int32_t* __restrict__ c_node_map,
                                  const double* __restrict__ xc, const uint8_t* __restrict__ f_cmask,
                                  double* __restrict__ x) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n_frow || !mg3_smooths(f_rowsim, depth, row, lev)) return;
  const int s = f_rowsim[row];
  const SimDev& F = fsims[s];
  const SimDev& C = csims[s];
  int ijk[3];
  node_ijk(F, f_active[row], ijk[0], ijk[1], ijk[2]);
  int lo[3], hi[3];
  double wl[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int v = ijk[a];
    if (a >= dim) { lo[a] = hi[a] = v; wl[a] = 1.0; }   // plane strain: the one z layer
    else if (v % 2 == 0) { lo[a] = hi[a] = v / 2; wl[a] = 1.0; }
    else { lo[a] = (v - 1) / 2; hi[a] = (v + 1) / 2; wl[a] = 0.5; }
  }
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int K = lo[2]; K <= hi[2]; ++K)
    for (int J = lo[1]; J <= hi[1]; ++J)
      for (int I = lo[0]; I <= hi[0]; ++I) {
        const int32_t cr = c_node_map[node_id(C, I, J, K)];
        if (cr < 0) continue;
        const double w = wl[0] * wl[1] * wl[2];
        a0 += w * xc[(int64_t)cr * 3];
        a1 += w * xc[(int64_t)cr * 3 + 1];
        a2 += w * xc[(int64_t)cr * 3 + 2];
      }
  if (!f_cmask[row * 3]) x[row * 3] += a0;
  if (!f_cmask[row * 3 + 1]) x[row * 3 + 1] += a1;
  if (!f_cmask[row * 3 + 2]) x[row * 3 + 2] += a2;
}

// Coarsest matrix, dense per sim: [A | I] of nmax x 2 nmax (row-major), the
// sim's rows first, from the rows of level lev whose simulation is solved
// there.  dense must be zeroed before.
__global__ void k_mg3_dense_fill(int64_t n_row, int lev, const int32_t* __restrict__ depth,
                                 const int32_t* __restrict__ row_sim,
                                 const int32_t* __restrict__ doff, const int32_t* __restrict__ rowptr,
                                 const int32_t* __restrict__ colind, const double* __restrict__ val, int nmax,
                                 double* __restrict__ dense) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n_row) return;
  const int s = row_sim[row];
  if (depth[s] != lev) return;
  const int r0 = doff[2 * s];
  double* M = dense + (int64_t)s * nmax * 2 * nmax;
  const int rl = (int)(row - r0);
  for (int32_t k = rowptr[row]; k < rowptr[row + 1]; ++k) {
    const int cl = colind[k] - r0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) M[(int64_t)(rl * 3 + a) * 2 * nmax + cl * 3 + b] = val[(int64_t)k * 9 + a * 3 + b];
  }
  for (int a = 0; a < 3; ++a) M[(int64_t)(rl * 3 + a) * 2 * nmax + nmax + rl * 3 + a] = 1.0;
}

// Gauss-Jordan with partial pivoting on [A | I] (one workgroup per sim, in
// global memory): afterwards the right half holds A^-1.  A zero pivot sets
// flag bit 16 and leaves that column unreduced.
constexpr int GJ3 = 1024;
__global__ void __launch_bounds__(GJ3) k_mg3_gauss_jordan(const int32_t* __restrict__ doff, int nmax,
                                                          double* __restrict__ dense, int32_t* __restrict__ flag) {
  __shared__ double fcol[MG3_DENSE_MAX];
  __shared__ double rv[GJ3];
  __shared__ int ri[GJ3];
  const int s = blockIdx.x;
  const int n = 3 * doff[2 * s + 1];
  double* M = dense + (int64_t)s * nmax * 2 * nmax;
  const int W = 2 * nmax, t = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    // pivot: largest |M[i][k]| over i >= k (ties to the smaller row)
    double best = -1.0;
    int bi = k;
    for (int i = k + t; i < n; i += GJ3) {
      const double v = fabs(M[(int64_t)i * W + k]);
      if (v > best) { best = v; bi = i; }
    }
    rv[t] = best;
    ri[t] = bi;
    __syncthreads();
    for (int off = GJ3 / 2; off > 0; off >>= 1) {
      if (t < off) {
        const double o = rv[t + off];
        const int oi = ri[t + off];
        if (o > rv[t] || (o == rv[t] && oi < ri[t])) { rv[t] = o; ri[t] = oi; }
      }
      __syncthreads();
    }
    const int p = ri[0];
    const double pv = M[(int64_t)p * W + k];
    __syncthreads();
    if (pv == 0.0) {
      if (t == 0) atomicOr(flag, 16);
      continue;
    }
    if (p != k)
      for (int j = t; j < W; j += GJ3) {
        const double a = M[(int64_t)k * W + j];
        M[(int64_t)k * W + j] = M[(int64_t)p * W + j];
        M[(int64_t)p * W + j] = a;
      }
    __syncthreads();
    const double ip = 1.0 / M[(int64_t)k * W + k];
    __syncthreads();   // every thread has read the pivot before row k is scaled
    for (int j = t; j < W; j += GJ3) M[(int64_t)k * W + j] *= ip;
    for (int i = t; i < n; i += GJ3) fcol[i] = M[(int64_t)i * W + k];
    __syncthreads();
    for (int e = t; e < n * W; e += GJ3) {
      const int i = e / W, j = e - i * W;
      if (i == k) continue;
      const double f = fcol[i];
      if (f != 0.0) M[(int64_t)i * W + j] -= f * M[(int64_t)k * W + j];
    }
    __syncthreads();
  }
}

// x = A^-1 b for the simulations whose coarsest level is lev (vectors of
// that level; per sim the right half of its dense block).
__global__ void k_mg3_dense_apply(int lev, const int32_t* __restrict__ depth, const int32_t* __restrict__ doff,
                                  int nmax, const double* __restrict__ dense, const double* __restrict__ b,
                                  double* __restrict__ x) {
  const int s = blockIdx.x;
  if (depth[s] != lev) return;
  const int r0 = doff[2 * s], n = 3 * doff[2 * s + 1];
  const double* M = dense + (int64_t)s * nmax * 2 * nmax;
  const double* bb = b + (int64_t)r0 * 3;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double a = 0.0;
    for (int j = 0; j < n; ++j) a += M[(int64_t)i * 2 * nmax + nmax + j] * bb[j];
    x[(int64_t)r0 * 3 + i] = a;
  }
}

}  // namespace mpm

using namespace mpm;

static unsigned nb256_3(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

static int level_lmax(mpm_ctx* c, int lev, const mpm_ctx* L, const double* val, const double* dinv, double* v,
                      double* w, double* lambda);

// Quadrature particles of level L (see the top of this file): per origin key
// its chunks of at most MG3_CHUNK sorted particles and its first quadrature
// particle, the non-empty keys, and the positions (and, plane strain, the
// fixed weights) of the quadrature particles.
static int build_quadrature(mpm_ctx* c, MgLevel* L, int dim) {
  mpm_ctx* sub = L->sub;
  const int64_t nk = sub->n_okeys;
  std::vector<int32_t> gs(nk + 1);
  HIPC(c, hipMemcpyAsync(gs.data(), sub->gstart.p, gs.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  const int ng = 1 << dim;
  const double g1 = 0.5 / std::sqrt(3.0);
  const double go[2] = {1.0 - g1, 1.0 + g1};   // Gauss points of [o + 1/2, o + 3/2] in cells
  std::vector<int32_t> ch, kc(nk + 1), pg(nk + 1), nek, qsim;
  std::vector<double> pos[3];
  int64_t npp = 0;
  int s = 0;
  for (int64_t k = 0; k < nk; ++k) {
    kc[k] = (int32_t)(ch.size() / 2);
    pg[k] = (int32_t)npp;
    for (int32_t p = gs[k]; p < gs[k + 1]; p += MG3_CHUNK) {
      ch.push_back(p);
      ch.push_back(std::min(MG3_CHUNK, gs[k + 1] - p));
    }
    if (gs[k + 1] == gs[k]) continue;
    while (s + 1 < sub->nsim && k >= sub->sims_h[s + 1].okey_base) ++s;
    const SimDev& S = sub->sims_h[s];
    const int64_t loc = k - S.okey_base;
    int o[3] = {(int)(loc % S.noa[0]) - 1, 0, 0};
    if (dim == 2) {
      o[1] = (int)(loc / S.noa[0]) - 1;
    } else {
      o[1] = (int)((loc / S.noa[0]) % S.noa[1]) - 1;
      o[2] = (int)(loc / ((int64_t)S.noa[0] * S.noa[1])) - 1;
    }
    nek.push_back((int32_t)k);
    for (int g = 0; g < ng; ++g) {
      for (int a = 0; a < dim; ++a) pos[a].push_back(S.x0[a] + S.h * (o[a] + go[(g >> a) & 1]));
      qsim.push_back(s);
    }
    npp += ng;
  }
  kc[nk] = (int32_t)(ch.size() / 2);
  pg[nk] = (int32_t)npp;
  L->n_chunks = (int64_t)(ch.size() / 2);
  L->npp = npp;
  L->n_nek = (int64_t)nek.size();
  const int stride = dim == 3 ? PTW3 : PU2;
  const int nent = dim == 3 ? PT3 : 49;
  if (L->chunk.ensure(std::max<size_t>(2, ch.size())) != hipSuccess || L->key_chunk.ensure(nk + 1) != hipSuccess ||
      L->pg.ensure(nk + 1) != hipSuccess || L->nek.ensure(std::max<size_t>(1, nek.size())) != hipSuccess ||
      L->qsim.ensure(std::max<int64_t>(1, npp)) != hipSuccess ||
      L->pxs.ensure(std::max<int64_t>(1, npp) * dim) != hipSuccess ||
      L->prec.ensure(std::max<int64_t>(1, npp) * stride) != hipSuccess ||
      L->part.ensure((size_t)std::max<int64_t>(1, L->n_chunks) * nent) != hipSuccess ||
      (dim == 2 && L->prgrp.ensure(std::max<int64_t>(1, sub->n_row) * 18) != hipSuccess))
    return c->fail(MPM_E_NOMEM, "multigrid quadrature allocation failed");
  if (!ch.empty())
    HIPC(c, hipMemcpyAsync(L->chunk.p, ch.data(), ch.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(L->key_chunk.p, kc.data(), kc.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(L->pg.p, pg.data(), pg.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  if (npp) {
    HIPC(c, hipMemcpyAsync(L->nek.p, nek.data(), nek.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIPC(c, hipMemcpyAsync(L->qsim.p, qsim.data(), qsim.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    for (int a = 0; a < dim; ++a)
      HIPC(c, hipMemcpyAsync(L->pxs.p + a * npp, pos[a].data(), npp * sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
  }
  if (dim == 2) {
    GUARD(launch_row_groups(sub, L->pg.p, L->prgrp.p));
    if (npp) {
      k_mgup_qweights<<<nb256_3(npp), 256, 0, c->stream>>>(npp, L->pxs.p, L->qsim.p, sub->sims.p, L->prec.p);
      LAUNCH_CHECK(c, "k_mgup_qweights");
    }
  } else if (npp) {
    k_mg3_qweights<<<nb256_3(npp), 256, 0, c->stream>>>(npp, L->pxs.p, L->qsim.p, sub->sims.p, L->prec.p);
    LAUNCH_CHECK(c, "k_mg3_qweights");
  }
  HIPC(c, hipStreamSynchronize(c->stream));   // the host tables above go out of scope
  return MPM_OK;
}

// Levels of the 3-D hierarchy for the current prepare of c (pb: the fine problem).
int mg3_build(mpm_ctx* c, const mpm_problem* pb) {
  if (!(c->dim == 3 && !c->up) && !(c->dim == 2 && c->up))
    return c->fail(MPM_E_INVALID, "the 3x3-block multigrid covers 3-D single-phase and plane-strain u-p problems");
  const int dim = c->dim;
  const int nsim = c->nsim;
  const int64_t np = c->np;
  if (c->mg_inv.ensure(std::max<int64_t>(1, np)) != hipSuccess ||
      c->mg_fine.ensure(std::max<int64_t>(1, 3 * c->n_row * 3)) != hipSuccess ||
      c->mg_sims.ensure(nsim) != hipSuccess)
    return c->fail(MPM_E_NOMEM, "multigrid allocation failed");
  if (np) {
    k_mg_inv_perm3<<<nb256_3(np), 256, 0, c->stream>>>(np, c->perm.p, c->mg_inv.p);
    LAUNCH_CHECK(c, "k_mg_inv_perm3");
  }
  std::vector<mpm_grid> grids(pb->grids, pb->grids + nsim);
  const mpm_ctx* finer = c;
  const uint8_t* fmask = pb->bc_mask;
  size_t nl = 0;
  for (int l = 1; l <= MG3_MAX_LEVELS; ++l) {
    int64_t worst = 0;
    bool shrinkable = false;
    for (int s = 0; s < nsim; ++s) {
      worst = std::max<int64_t>(worst, 3 * (finer->sim_row_start[s + 1] - finer->sim_row_start[s]));
      for (int k = 0; k < dim; ++k) shrinkable = shrinkable || grids[s].ncell[k] > 1;
    }
    if (worst <= MG3_DENSE_MAX || !shrinkable) break;
    for (int s = 0; s < nsim; ++s) {
      grids[s].h *= 2.0;
      for (int k = 0; k < dim; ++k) grids[s].ncell[k] = std::max(1, (grids[s].ncell[k] + 1) / 2);
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
    std::vector<SimDev> cs(nsim);
    int64_t n_cnodes = 0;
    for (int s = 0; s < nsim; ++s) {
      SimDev& S = cs[s];
      S = SimDev{};
      for (int k = 0; k < dim; ++k) {
        S.n[k] = grids[s].ncell[k];
        S.nna[k] = grids[s].ncell[k] + 3;
        S.noa[k] = grids[s].ncell[k] + 1;
      }
      if (dim == 2) { S.n[2] = 0; S.nna[2] = 1; S.noa[2] = 1; }
      S.node_base = n_cnodes;
      n_cnodes += (int64_t)S.nna[0] * S.nna[1] * S.nna[2];
    }
    if (L->mask.ensure(std::max<int64_t>(1, 3 * n_cnodes)) != hipSuccess ||
        c->mg_zero.ensure(std::max<size_t>(c->mg_zero.n, (size_t)std::max<int64_t>(1, 3 * n_cnodes))) != hipSuccess)
      return c->fail(MPM_E_NOMEM, "multigrid mask allocation failed");
    HIPC(c, hipMemsetAsync(c->mg_zero.p, 0, c->mg_zero.n * sizeof(double), c->stream));
    HIPC(c, hipMemcpyAsync(c->mg_sims.p, cs.data(), nsim * sizeof(SimDev), hipMemcpyHostToDevice, c->stream));
    k_mg3_mask<<<nb256_3(n_cnodes), 256, 0, c->stream>>>(n_cnodes, nsim, dim, c->mg_sims.p, finer->sims.p, fmask,
                                                         L->mask.p);
    LAUNCH_CHECK(c, "k_mg3_mask");
    mpm_problem cp = *pb;
    cp.mat.shape = 0;   // coarse levels are rediscretized with quadratic B-splines (a preconditioner only)
    cp.grids = L->grids.data();
    cp.bc_mask = L->mask.p;
    cp.bc_value = c->mg_zero.p;
    cp.react_mask = nullptr;
    int rc = mpm_prepare_impl(sub, &cp, nullptr, nullptr, nullptr);
    if (rc) return c->fail(rc, "multigrid level " + std::to_string(l) + ": " + sub->err);
    if (L->pmap.ensure(std::max<int64_t>(1, np)) != hipSuccess ||
        L->vec.ensure(std::max<int64_t>(1, 5 * sub->n_row * 3)) != hipSuccess ||
        sub->val.ensure(std::max<int64_t>(1, sub->nnzb * 9)) != hipSuccess)
      return c->fail(MPM_E_NOMEM, "multigrid level allocation failed");
    if (np) {
      k_mg_pmap3<<<nb256_3(np), 256, 0, c->stream>>>(np, sub->perm.p, c->mg_inv.p, L->pmap.p);
      LAUNCH_CHECK(c, "k_mg_pmap3");
    }
    GUARD(build_quadrature(c, L, dim));
    finer = sub;
    fmask = L->mask.p;
    nl = l;
  }
  while (c->mgl.size() > nl) { mg_level_release(c->mgl.back()); c->mgl.pop_back(); }
  c->mg_tail_first = -1;
  // per sim: its coarsest level (the first with at most MG3_DENSE_MAX
  // unknowns, else the last) and its rows there
  std::vector<int32_t> doff(2 * nsim);
  c->mg3_depth_h.assign(nsim, (int32_t)nl);
  int nmax = 3;
  for (int s = 0; s < nsim; ++s) {
    for (size_t l = 0; l <= nl; ++l) {
      const mpm_ctx* C = l ? c->mgl[l - 1]->sub : c;
      if (3 * (C->sim_row_start[s + 1] - C->sim_row_start[s]) <= MG3_DENSE_MAX || l == nl) {
        c->mg3_depth_h[s] = (int32_t)l;
        doff[2 * s] = (int32_t)C->sim_row_start[s];
        doff[2 * s + 1] = (int32_t)(C->sim_row_start[s + 1] - C->sim_row_start[s]);
        break;
      }
    }
    nmax = std::max(nmax, 3 * doff[2 * s + 1]);
  }
  if (nmax > MG3_DENSE_MAX) return c->fail(MPM_E_INVALID, "multigrid coarsest level too large for the dense solve");
  c->mg_nmax = nmax;
  if (c->mg_doff.ensure(2 * nsim) != hipSuccess || c->mg3_depth.ensure(nsim) != hipSuccess ||
      c->mg_dense.ensure((size_t)nsim * 2 * nmax * nmax) != hipSuccess)
    return c->fail(MPM_E_NOMEM, "multigrid dense allocation failed");
  HIPC(c, hipMemcpyAsync(c->mg_doff.p, doff.data(), doff.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(c->mg3_depth.p, c->mg3_depth_h.data(), nsim * sizeof(int32_t), hipMemcpyHostToDevice,
                         c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  ++c->mg_gen;
  c->mg_ready = true;
  return MPM_OK;
}

// Per Newton iteration, after the fine Jacobian (tangent records in
// c->pdat3, u-p: c->pdat) and its block-Jacobi inverse: level matrices,
// inverses and the coarsest inverse.
int mg3_setup(mpm_ctx* c) {
  for (MgLevel* L : c->mgl) {
    mpm_ctx* sub = L->sub;
    // quadrature particle tables: the finest tables summed per origin of this level
    const int stride = c->up ? PU2 : PTW3, nent = c->up ? 49 : PT3, ng = c->up ? 4 : 8;
    if (L->n_chunks) {
      k_mg3_chunk_sum<<<(unsigned)L->n_chunks, 128, 0, c->stream>>>(L->n_chunks, L->chunk.p, L->pmap.p,
                                                                   c->up ? c->pdat.p : c->pdat3.p, stride, nent,
                                                                   L->part.p);
      LAUNCH_CHECK(c, "k_mg3_chunk_sum");
    }
    if (L->n_nek) {
      k_mg3_qrec<<<(unsigned)L->n_nek, 128, 0, c->stream>>>(L->n_nek, L->nek.p, L->key_chunk.p, L->part.p, nent,
                                                            L->pg.p, ng, stride, L->prec.p);
      LAUNCH_CHECK(c, "k_mg3_qrec");
    }
    int rc = c->up ? launch_jac2up_records(sub, L->prec.p, sub->val.p, true, L->prgrp.p)
                   : launch_jac3_lines(sub, L->prec.p, nullptr, sub->val.p, true, L->pg.p);
    if (!rc) rc = launch_bj_inv(sub, sub->val.p);
    if (rc) return c->fail(rc, "multigrid level setup: " + sub->err);
  }
  // lambda_max(D^-1 A) of every smoothed level and sim (the level's own
  // vectors as scratch), then the Chebyshev coefficients of every step
  const size_t nl = c->mgl.size();
  const int nsim = c->nsim;
  if (nl) {
    int64_t most_rows = c->n_row;
    for (MgLevel* L : c->mgl) most_rows = std::max(most_rows, L->sub->n_row);
    if (c->mg3_lam.ensure(nl * nsim) != hipSuccess || c->mg3_inv.ensure(nsim) != hipSuccess ||
        c->mg3_part.ensure(std::max<int64_t>(1, most_rows)) != hipSuccess ||
        c->mg3_coef.ensure(nl * MG3_DEG * nsim * 2) != hipSuccess)
      return c->fail(MPM_E_NOMEM, "multigrid allocation failed");
    for (size_t l = 0; l < nl; ++l) {
      const mpm_ctx* L = l == 0 ? c : c->mgl[l - 1]->sub;
      const double* val = l == 0 ? c->val.p : L->val.p;
      const double* dinv = l == 0 ? c->dinv.p : L->dinv.p;
      const int64_t nv = L->n_row * 3;
      double* v = l == 0 ? c->mg_fine.p : c->mgl[l - 1]->vec.p;
      GUARD(level_lmax(c, (int)l, L, val, dinv, v, v + nv, c->mg3_lam.p + l * nsim));
    }
    c->mg3_lmax.assign(nl * nsim, 1.0);
    HIPC(c, hipMemcpyAsync(c->mg3_lmax.data(), c->mg3_lam.p, nl * nsim * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    HIPC(c, hipStreamSynchronize(c->stream));
    // step k: x_k = x_{k-1} + d_k, d_k = c0 d_{k-1} + c1 D^-1 r (the three-term
    // Chebyshev recurrence on [lo, hi] = [MG3_LO, MG3_HI] x lambda_max)
    std::vector<double> coef(nl * MG3_DEG * nsim * 2);
    for (size_t l = 0; l < nl; ++l)
      for (int q = 0; q < nsim; ++q) {
        const double lmax = c->mg3_lmax[l * nsim + q];
        const double lo = MG3_LO * lmax, hi = (c->up ? MG3_HI_UP : MG3_HI_3D) * lmax;
        const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
        double rho = 1.0 / sigma;
        for (int k = 0; k < MG3_DEG; ++k) {
          double c0 = 0.0, c1 = 1.0 / theta;
          if (k > 0) {
            const double rn = 1.0 / (2.0 * sigma - rho);
            c0 = rn * rho;
            c1 = 2.0 * rn / delta;
            rho = rn;
          }
          double* e = coef.data() + ((l * MG3_DEG + k) * nsim + q) * 2;
          e[0] = c0;
          e[1] = c1;
        }
      }
    HIPC(c, hipMemcpyAsync(c->mg3_coef.p, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
    HIPC(c, hipStreamSynchronize(c->stream));   // coef goes out of scope
  }
  // every sim's dense block from its own coarsest level
  const int nmax = c->mg_nmax;
  HIPC(c, hipMemsetAsync(c->mg_dense.p, 0, (size_t)c->nsim * 2 * nmax * nmax * sizeof(double), c->stream));
  for (size_t l = 0; l <= c->mgl.size(); ++l) {
    if (std::find(c->mg3_depth_h.begin(), c->mg3_depth_h.end(), (int32_t)l) == c->mg3_depth_h.end()) continue;
    const mpm_ctx* C = l == 0 ? c : c->mgl[l - 1]->sub;
    const double* Cval = l == 0 ? c->val.p : C->val.p;
    if (!C->n_row) continue;
    k_mg3_dense_fill<<<nb256_3(C->n_row), 256, 0, c->stream>>>(C->n_row, (int)l, c->mg3_depth.p, C->row_sim.p,
                                                               c->mg_doff.p, C->rowptr.p, C->colind.p, Cval, nmax,
                                                               c->mg_dense.p);
    LAUNCH_CHECK(c, "k_mg3_dense_fill");
  }
  k_mg3_gauss_jordan<<<(unsigned)c->nsim, GJ3, 0, c->stream>>>(c->mg_doff.p, nmax, c->mg_dense.p, c->flag.p);
  LAUNCH_CHECK(c, "k_mg3_gauss_jordan");
  return MPM_OK;
}

static unsigned rows_grid(int64_t n_row) { return (unsigned)((n_row * MG3_LPR + 255) / 256); }

// Chebyshev smoothing of level lev (context L) from x_in (null: 0) into x,
// with every sim's own coefficients; d is scratch.
static int cheb3(mpm_ctx* c, int lev, const mpm_ctx* L, const double* val, const double* dinv, const double* b,
                 double* x, double* xs, double* d, bool from_zero) {
  const int64_t n_row = L->n_row;
  if (!n_row) return MPM_OK;
  // step k writes x when DEG-1-k is even, else xs, so the last lands in x;
  // no step reads the vector it writes (the products need the old iterate)
  const double* xin = nullptr;
  if (!from_zero) {
    if (MG3_DEG % 2 == 1) {   // the first step writes x: start from a copy
      HIPC(c, hipMemcpyAsync(xs, x, n_row * 3 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      xin = xs;
    } else {
      xin = x;
    }
  }
  for (int k = 0; k < MG3_DEG; ++k) {
    double* out = ((MG3_DEG - 1 - k) % 2 == 0) ? x : xs;
    k_mg3_cheb<<<rows_grid(n_row), 256, 0, c->stream>>>(n_row, lev, L->row_sim.p, c->mg3_depth.p, L->rowptr.p,
                                                         L->colind.p, val, dinv, b, xin, out, d,
                                                         c->mg3_coef.p + ((size_t)lev * MG3_DEG + k) * c->nsim * 2,
                                                         k == 0);
    LAUNCH_CHECK(c, "k_mg3_cheb");
    xin = out;
  }
  return MPM_OK;
}

// lambda_max(D^-1 A) of level lev's smoothed rows, per sim, by power
// iteration (deterministic sums, no host round trip): lambda[s] on the device.
static int level_lmax(mpm_ctx* c, int lev, const mpm_ctx* L, const double* val, const double* dinv, double* v,
                      double* w, double* lambda) {
  const int64_t n_row = L->n_row;
  if (!n_row) {
    std::vector<double> one(c->nsim, 1.0);
    HIPC(c, hipMemcpyAsync(lambda, one.data(), one.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPC(c, hipStreamSynchronize(c->stream));
    return MPM_OK;
  }
  const int64_t nv = n_row * 3;
  k_mg3_scale<<<nb256_3(nv), 256, 0, c->stream>>>(nv, L->row_sim.p, L->sims.p, nullptr, nullptr, v);
  LAUNCH_CHECK(c, "k_mg3_scale");
  for (int it = 0; it < MG3_POWER; ++it) {
    k_mg3_pow<<<rows_grid(n_row), 256, 0, c->stream>>>(n_row, lev, L->row_sim.p, c->mg3_depth.p, L->rowptr.p,
                                                        L->colind.p, val, dinv, v, w, c->mg3_part.p);
    LAUNCH_CHECK(c, "k_mg3_pow");
    k_mg3_pow_sim<<<(unsigned)c->nsim, 256, 0, c->stream>>>(n_row, c->nsim, L->sims.p, c->mg3_part.p, c->mg3_inv.p,
                                                            lambda, it == 0);
    LAUNCH_CHECK(c, "k_mg3_pow_sim");
    // lambda = ||D^-1 A v|| with ||v|| = 1 (after the first step)
    k_mg3_scale<<<nb256_3(nv), 256, 0, c->stream>>>(nv, L->row_sim.p, L->sims.p, w, c->mg3_inv.p, v);
    LAUNCH_CHECK(c, "k_mg3_scale");
  }
  return MPM_OK;
}

// out = M^-1 b on level l: the dense solve of the simulations whose
// coarsest level is l, a V-cycle for those with deeper ones.
static int vcycle3(mpm_ctx* c, size_t l, const double* b, double* out) {
  const size_t nl = c->mgl.size();
  const std::vector<int32_t>& dep = c->mg3_depth_h;
  if (std::find(dep.begin(), dep.end(), (int32_t)l) != dep.end()) {
    k_mg3_dense_apply<<<(unsigned)c->nsim, 256, 0, c->stream>>>((int)l, c->mg3_depth.p, c->mg_doff.p, c->mg_nmax,
                                                               c->mg_dense.p, b, out);
    LAUNCH_CHECK(c, "k_mg3_dense_apply");
  }
  if (l == nl) return MPM_OK;
  const mpm_ctx* ctx = l == 0 ? c : c->mgl[l - 1]->sub;
  const double* val = l == 0 ? c->val.p : ctx->val.p;
  const double* dinv = l == 0 ? c->dinv.p : ctx->dinv.p;
  const int64_t nv = ctx->n_row * 3;
  double* y = l == 0 ? c->mg_fine.p : c->mgl[l - 1]->vec.p;            // iterate partner
  double* r = l == 0 ? c->mg_fine.p + nv : c->mgl[l - 1]->vec.p + nv;  // residual
  double* d = l == 0 ? c->mg_fine.p + 2 * nv : c->mgl[l - 1]->vec.p + 4 * nv;   // Chebyshev direction
  GUARD(cheb3(c, (int)l, ctx, val, dinv, b, out, y, d, true));
  if (ctx->n_row) {
    k_mg3_resid<<<rows_grid(ctx->n_row), 256, 0, c->stream>>>(ctx->n_row, (int)l, ctx->row_sim.p, c->mg3_depth.p,
                                                              ctx->rowptr.p, ctx->colind.p, val, b, out, r);
    LAUNCH_CHECK(c, "k_mg3_resid");
  }
  MgLevel* CL = c->mgl[l];
  const mpm_ctx* C = CL->sub;
  double* xc = CL->vec.p + 2 * C->n_row * 3;
  double* bc = CL->vec.p + 3 * C->n_row * 3;
  if (C->n_row) {
    k_mg3_restrict<<<nb256_3(C->n_row), 256, 0, c->stream>>>(C->n_row, c->dim, (int)l, c->mg3_depth.p,
                                                             C->active_nodes.p, C->row_sim.p, C->sims.p, ctx->sims.p,
                                                             ctx->node_map.p, r, C->cmask.p, bc);
    LAUNCH_CHECK(c, "k_mg3_restrict");
  }
  GUARD(vcycle3(c, l + 1, bc, xc));
  if (ctx->n_row) {
    k_mg3_prolong_add<<<nb256_3(ctx->n_row), 256, 0, c->stream>>>(ctx->n_row, c->dim, (int)l, c->mg3_depth.p,
                                                                  ctx->active_nodes.p, ctx->row_sim.p, ctx->sims.p,
                                                                  C->sims.p, C->node_map.p, xc, ctx->cmask.p, out);
    LAUNCH_CHECK(c, "k_mg3_prolong_add");
  }
  GUARD(cheb3(c, (int)l, ctx, val, dinv, b, out, y, d, false));
  return MPM_OK;
}

int mg3_vcycle(mpm_ctx* c, const double* b, double* x) { return vcycle3(c, 0, b, x); }
