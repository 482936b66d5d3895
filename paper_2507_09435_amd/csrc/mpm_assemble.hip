// Residual, localized Jacobian and particle update kernels (one thread per
// particle, particles sorted by stencil origin).
//
// Residual (Sec. 2.2): f_int,i = sum_p V0 P_p grad w_ip with P = tau dF^-T,
// r = f_int - f_ext.  Jacobian (Sec. 3.2): every particle owns a dense local
// block over its 3^d stencil nodes; here the block is the contraction
//   K_ab = V0 (out-weights of a) . T . (in-weights of b)
// of the particle's tangent table T (derivatives of its stress outputs with
// respect to dF and, for u-p, to p and grad p), obtained by forward-mode
// passes of the same stress code, then scattered into the BSR pattern.
#include "mpm_internal.hpp"

namespace mpm {

struct AsmArgs {
  int64_t np;
  int nd, up, dp, match, nsim;
  const double *xs, *vs, *Fs, *bes, *Es, *phis;   // sorted SoA (Es/phis may be null)
  const int32_t* psim;
  const SimDev* sims;
  const int32_t* node_map;
  double E, nu, phi, c, psi, apex_reg;
  double biot, mob, dt, rho_f, g[3];
};

__device__ __forceinline__ UpPar up_par(const AsmArgs& A) {
  return UpPar{A.biot, A.mob, A.dt, A.rho_f, {A.g[0], A.g[1], A.g[2]}};
}

// ------------------------------------------------------ per-particle load ---
template <int DIM>
struct PLoad {
  Stencil<DIM> st;
  int32_t row[Stencil<DIM>::NN];
  double dF[DIM][DIM];
  double pp, gp[DIM];
  double v0, Jn;
  double E, phi;
};

template <int DIM>
__device__ __forceinline__ void load_particle(const AsmArgs& A, int64_t i, const double* __restrict__ du, PLoad<DIM>& L) {
  const SimDev& S = A.sims[A.psim[i]];
  make_stencil<DIM>(S, A.xs, A.np, i, L.st);
#pragma unroll
  for (int r = 0; r < DIM; ++r)
#pragma unroll
    for (int c = 0; c < DIM; ++c) L.dF[r][c] = (r == c) ? 1.0 : 0.0;
  L.pp = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) L.gp[k] = 0.0;
  const int nd = A.nd;
  if constexpr (DIM == 2) {
    // every node-map load, then every increment load, is issued before the
    // first sum (the u-p choice is made once, outside the node loop); the
    // sums then take the nodes in order, as in the loop below
    constexpr int NN = Stencil<2>::NN;
    int32_t rr[NN];
#pragma unroll
    for (int a = 0; a < NN; ++a) rr[a] = A.node_map[L.st.node(S, a)];
    double uu[NN][3];
    if (A.up) {
#pragma unroll
      for (int a = 0; a < NN; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) uu[a][c] = du[(int64_t)rr[a] * 3 + c];
    } else {
#pragma unroll
      for (int a = 0; a < NN; ++a) {
        uu[a][0] = du[(int64_t)rr[a] * 2];
        uu[a][1] = du[(int64_t)rr[a] * 2 + 1];
        uu[a][2] = 0.0;
      }
    }
#pragma unroll
    for (int a = 0; a < NN; ++a) {
      L.row[a] = rr[a];
      double g[2];
      L.st.grad(a, g);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double uq = uu[a][q];
#pragma unroll
        for (int k = 0; k < 2; ++k) L.dF[q][k] += uq * g[k];
      }
      if (A.up) {
        const double pa = uu[a][2];
        L.pp += L.st.weight(a) * pa;
#pragma unroll
        for (int k = 0; k < 2; ++k) L.gp[k] += pa * g[k];
      }
    }
  } else {
    // one z-layer of nine nodes at a time: its node-map loads, then its
    // increment loads, then the sums, all unrolled (the stencil arrays stay
    // in registers)
#pragma unroll
    for (int az = 0; az < 3; ++az) {
      int32_t rr[9];
#pragma unroll
      for (int a9 = 0; a9 < 9; ++a9) rr[a9] = A.node_map[L.st.node(S, a9 + 9 * az)];
      double uu[9][3];
#pragma unroll
      for (int a9 = 0; a9 < 9; ++a9)
#pragma unroll
        for (int q = 0; q < 3; ++q) uu[a9][q] = du[(int64_t)rr[a9] * nd + q];
#pragma unroll
      for (int a9 = 0; a9 < 9; ++a9) {
        const int a = a9 + 9 * az;
        L.row[a] = rr[a9];
        double g[DIM];
        L.st.grad(a, g);
#pragma unroll
        for (int q = 0; q < DIM; ++q)
#pragma unroll
          for (int k = 0; k < DIM; ++k) L.dF[q][k] += uu[a9][q] * g[k];
      }
    }
  }
  L.v0 = A.vs[i];
  if (DIM == 2 && A.up) {
    L.Jn = A.Fs[0 * A.np + i] * A.Fs[3 * A.np + i] - A.Fs[1 * A.np + i] * A.Fs[2 * A.np + i];
  } else {
    L.Jn = 1.0;
  }
  L.E = A.Es ? A.Es[i] : A.E;
  L.phi = A.phis ? A.phis[i] : A.phi;
}

// The 3-D load of load_particle without the stencil's rows (L.row is left
// unset), for kernels that evaluate the stress only: the z-layers are taken
// one at a time in a loop, so at most one layer's nine node-map and 27
// increment loads are in flight and the register budget leaves room for a
// second wave per SIMD.  Same sums in the same order as load_particle<3>.
__device__ __forceinline__ void load_particle3_lean(const AsmArgs& A, int64_t i, const double* __restrict__ du,
                                                    PLoad<3>& L) {
  const SimDev& S = A.sims[A.psim[i]];
  make_stencil<3>(S, A.xs, A.np, i, L.st);
  double w0[3], w1[3], d0[3], d1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) { w0[a] = L.st.w[0][a]; w1[a] = L.st.w[1][a]; d0[a] = L.st.dw[0][a]; d1[a] = L.st.dw[1][a]; }
  double dF[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) dF[r][c] = (r == c) ? 1.0 : 0.0;
  const int nd = A.nd;
  const int64_t sy = S.nna[0], sz = (int64_t)S.nna[0] * S.nna[1];
  const int64_t base = S.node_base + (L.st.o[0] + 1) + sy * (L.st.o[1] + 1) + sz * (L.st.o[2] + 1);
  const double wz3[3] = {L.st.w[2][0], L.st.w[2][1], L.st.w[2][2]};
  const double dz3[3] = {L.st.dw[2][0], L.st.dw[2][1], L.st.dw[2][2]};
#pragma unroll 1
  for (int az = 0; az < 3; ++az) {
    const double wz = az == 0 ? wz3[0] : (az == 1 ? wz3[1] : wz3[2]);
    const double dwz = az == 0 ? dz3[0] : (az == 1 ? dz3[1] : dz3[2]);
    int32_t rr[9];
#pragma unroll
    for (int a9 = 0; a9 < 9; ++a9) rr[a9] = A.node_map[base + sz * az + (a9 % 3) + sy * (a9 / 3)];
    double uu[9][3];
#pragma unroll
    for (int a9 = 0; a9 < 9; ++a9)
#pragma unroll
      for (int q = 0; q < 3; ++q) uu[a9][q] = du[(int64_t)rr[a9] * nd + q];
#pragma unroll
    for (int a9 = 0; a9 < 9; ++a9) {
      const int ax = a9 % 3, ay = a9 / 3;
      const double g0 = d0[ax] * w1[ay] * wz, g1 = w0[ax] * d1[ay] * wz, g2 = w0[ax] * w1[ay] * dwz;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        dF[q][0] += uu[a9][q] * g0;
        dF[q][1] += uu[a9][q] * g1;
        dF[q][2] += uu[a9][q] * g2;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) L.dF[r][c] = dF[r][c];
  L.pp = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) L.gp[k] = 0.0;
  L.v0 = A.vs[i];
  L.Jn = 1.0;
  L.E = A.Es ? A.Es[i] : A.E;
  L.phi = A.phis ? A.phis[i] : A.phi;
}

__device__ __forceinline__ Sym2<double> load_be2(const AsmArgs& A, int64_t i) {
  return Sym2<double>{A.bes[0 * A.np + i], A.bes[1 * A.np + i], A.bes[2 * A.np + i], A.bes[3 * A.np + i]};
}
__device__ __forceinline__ Sym3<double> load_be3(const AsmArgs& A, int64_t i) {
  Sym3<double> b;
#pragma unroll
  for (int t = 0; t < 6; ++t) b.a[t] = A.bes[t * A.np + i];
  return b;
}

// r_raw = f_int - f_ext; r = r_raw with constrained unknowns zeroed.  Per-row-
// block partials: [0] = ||r||^2, [1] = sum of r_raw over the reaction mask.
__global__ void __launch_bounds__(64) k_res_final(const RowBlock* __restrict__ blocks, int nd,
                                                  const double* __restrict__ fint, const double* __restrict__ fext,
                                                  const uint8_t* __restrict__ cmask, const uint8_t* __restrict__ rmask,
                                                  double* __restrict__ r, double* __restrict__ r_raw,
                                                  double* __restrict__ part) {
  RowBlock b = blocks[blockIdx.x];
  int64_t row = b.row0 + threadIdx.x;
  double sq = 0.0, re = 0.0;
  if (row < b.row1) {
    for (int c = 0; c < nd; ++c) {
      int64_t k = row * nd + c;
      double raw = fint[k] - fext[k];
      if (r_raw) r_raw[k] = raw;
      if (rmask[k]) re += raw;
      double v = cmask[k] ? 0.0 : raw;
      if (r) r[k] = v;
      sq += v * v;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    sq += __shfl_down(sq, off, 64);
    re += __shfl_down(re, off, 64);
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x * NQ + 0] = sq;
    part[blockIdx.x * NQ + 1] = re;
  }
}

// Per sim: sum the row-block partials in block order (deterministic).
__global__ void __launch_bounds__(64) k_sim_sum(int nsim, const int32_t* __restrict__ blk_first,
                                                const double* __restrict__ part, int q, double* __restrict__ out,
                                                int out_stride, int out_off) {
  const int s = blockIdx.x;   // one wave per sim, fixed lane assignment and reduction order
  const int b1 = blk_first[s + 1];
  double acc = 0.0;
  // a lane adds its blocks b, b + 64, ... in order; eight loads are issued before their adds
  for (int b0 = blk_first[s] + (int)threadIdx.x; b0 < b1; b0 += 8 * 64) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = b0 + 64 * u < b1 ? part[(b0 + 64 * u) * NQ + q] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b0 + 64 * u < b1) acc += v[u];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (threadIdx.x == 0) out[s * out_stride + out_off] = acc;
}

// k_sim_sum for the residual's two partial sums (||r||^2 and the reaction)
// in one launch, each in the same lanes and order as k_sim_sum.
__global__ void __launch_bounds__(64) k_sim_sum_res(const int32_t* __restrict__ blk_first,
                                                    const double* __restrict__ part, double* __restrict__ out) {
  const int s = blockIdx.x;
  const int b1 = blk_first[s + 1];
  double a0 = 0.0, a1 = 0.0;
  for (int b0 = blk_first[s] + (int)threadIdx.x; b0 < b1; b0 += 8 * 64) {
    double v0[8], v1[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = b0 + 64 * u < b1;
      v0[u] = in ? part[(b0 + 64 * u) * NQ + 0] : 0.0;
      v1[u] = in ? part[(b0 + 64 * u) * NQ + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b0 + 64 * u < b1) {
        a0 += v0[u];
        a1 += v1[u];
      }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a0 += __shfl_xor(a0, off, 64);
    a1 += __shfl_xor(a1, off, 64);
  }
  if (threadIdx.x == 0) {
    out[s * 16 + 0] = a0;
    out[s * 16 + 1] = a1;
  }
}

// ----------------------------------------------------------- Jacobian ------
// Column q of the tangent table of one 2-D particle: derivatives of the
// outputs (P (4), then for u-p s1 and vv (2)) with respect to input q
// (dF (4), then for u-p p and grad p (2)), by one forward-mode pass.
template <int NIO>
__device__ __forceinline__ void tangent2_col(const AsmArgs& A, const PLoad<2>& L, const Sym2<double>& be, int q,
                                             double Tc[NIO]) {
  // the material constants carry no derivative here
  const Mat<double> m = make_mat<double>(L.E, A.nu, L.phi, A.c, A.psi, A.dp, A.match, A.apex_reg);
  UpPar u = up_par(A);
  dnum F[2][2];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < 2; ++c) F[r][c] = dnum(L.dF[r][c], q == r * 2 + c ? 1.0 : 0.0);
  dnum pp(L.pp, q == 4 ? 1.0 : 0.0);
  dnum gp[2] = {dnum(L.gp[0], q == 5 ? 1.0 : 0.0), dnum(L.gp[1], q == 6 ? 1.0 : 0.0)};
  Sym2<dnum> bd{dnum(be.xx), dnum(be.yy), dnum(be.xy), dnum(be.zz)};
  Out2<dnum> o;
  mech2<dnum, double>(m, F, bd, dnum(L.Jn), NIO == 7, u, pp, gp, o, nullptr);
  Tc[0] = o.P[0][0].d; Tc[1] = o.P[0][1].d; Tc[2] = o.P[1][0].d; Tc[3] = o.P[1][1].d;
  if constexpr (NIO == 7) { Tc[4] = o.s1.d; Tc[5] = o.vv[0].d; Tc[6] = o.vv[1].d; }
}

// 2-D single-phase Jacobian without atomics, in two deterministic passes.
// k_tan2: one record per particle (sorted order): V0 * tangent table (dP/dF,
// 4x4, output-major) and its stencil's weights and derivatives per axis.
// k_jac2_rows: every BSR block (a, b) is the sum, in origin order, of the
// group blocks of the (at most nine) stencil groups holding both nodes,
// written once (no clearing, no atomics).

__global__ void __launch_bounds__(256) k_tan2(AsmArgs A, const double* __restrict__ du, double* __restrict__ pdat) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = gid >> 2;
  const int q = (int)(gid & 3);
  if (i >= A.np) return;
  PLoad<2> L;
  load_particle<2>(A, i, du, L);
  double Tc[4];
  tangent2_col<4>(A, L, load_be2(A, i), q, Tc);
  double* P = pdat + i * PD2;
#pragma unroll
  for (int o = 0; o < 4; ++o) P[o * 4 + q] = L.v0 * Tc[o];
#pragma unroll
  for (int a = 0; a < 3; ++a)   // lane a < 3 stores entry a (constant indices keep the stencil in registers)
    if (q == a) {
      P[16 + a] = L.st.w[0][a];
      P[19 + a] = L.st.dw[0][a];
      P[22 + a] = L.st.w[1][a];
      P[25 + a] = L.st.dw[1][a];
    }
}

__device__ __forceinline__ double sel3(int i, double v0, double v1, double v2) {
  return i == 0 ? v0 : (i == 1 ? v1 : v2);
}


// Fused 2-D single-phase Jacobian from the tangent records: a workgroup of
// JR rows with 16 lanes each.  Lane q < 9 of row a takes the q-th stencil
// group that may hold node a (its particle range from the row group table)
// and accumulates, over its particles in order, the nine 2x2 blocks (a, b)
// for the group's local nodes b, into LDS.  Then each BSR block (a, b) of the
// JR rows sums the groups holding both nodes, in group order, and takes
// Dirichlet rows and columns as the identity's.  Every group block is formed
// once, as by a group-block pass followed by a block gather, without the
// group blocks' round trip through HBM.  The second pass needs only the
// slot and constraint tables of its rows, loaded before the first pass, so
// no chain of dependent global loads is left on the way.
constexpr int JR = 16;   // rows per workgroup (16 lanes each)
constexpr int JB = (JR * 25 + 255) / 256;   // stencil offsets per thread in the block pass
__global__ void __launch_bounds__(256) k_jac2_rows(int64_t n_row, const int32_t* __restrict__ rgrp,
                                                  const double* __restrict__ pdat,
                                                  const int32_t* __restrict__ rowptr,
                                                  const int8_t* __restrict__ slot,
                                                  const uint8_t* __restrict__ bcode, double* __restrict__ val) {
  __shared__ double part[JR][9][9 * 4];   // [row][group q][local node b][2x2]
  const int rl = threadIdx.x / 16, q = threadIdx.x % 16;
  const int64_t row0 = (int64_t)blockIdx.x * JR;
  // block pass: thread t takes stencil offsets t and t + 256 of the JR rows
  // (independent loads, in flight during the first pass)
  int32_t sl[JB], rp[JB];
  uint32_t code[JB];
#pragma unroll
  for (int h = 0; h < JB; ++h) {
    const int t = threadIdx.x + 256 * h;
    const int64_t row = row0 + t / 25;
    sl[h] = -1;
    rp[h] = 0;
    code[h] = 0;
    if (t < JR * 25 && row < n_row) {
      sl[h] = slot[row * 25 + t % 25];
      rp[h] = rowptr[row];
      if (bcode) code[h] = bcode[row * 25 + t % 25];
    }
  }
  {
    const int64_t row = row0 + rl;
    if (row < n_row && q < 9) {
      const int p0 = rgrp[(row * 9 + q) * 2], p1 = rgrp[(row * 9 + q) * 2 + 1];
      const int ax = 2 - q % 3, ay = 2 - q / 3;   // node a's place in the group's 3x3 stencil
      double K[9][4];
#pragma unroll
      for (int lb = 0; lb < 9; ++lb)
#pragma unroll
        for (int e = 0; e < 4; ++e) K[lb][e] = 0.0;
      for (int p = p0; p < p1; ++p) {
        const double* P = pdat + (int64_t)p * PD2;
        double T[16], w[12];
#pragma unroll
        for (int k = 0; k < 16; ++k) T[k] = P[k];
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] = P[16 + k];
        // w: wx 0..2, dwx 3..5, wy 6..8, dwy 9..11; grad w_n = (dwx wy, wx dwy)
        const double ga0 = sel3(ax, w[3], w[4], w[5]) * sel3(ay, w[6], w[7], w[8]);
        const double ga1 = sel3(ax, w[0], w[1], w[2]) * sel3(ay, w[9], w[10], w[11]);
        // K_ab[r][c] = sum_ij ga_i T[(2r+i)4 + 2c+j] gb_j: contract node a's side once,
        // U[r][c][j] = sum_i ga_i T[(2r+i)4 + 2c+j], then two fma per entry and node b
        double U[2][2][2];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              U[r][c][j] = fma(ga1, T[(2 * r + 1) * 4 + 2 * c + j], ga0 * T[(2 * r) * 4 + 2 * c + j]);
#pragma unroll
        for (int lb = 0; lb < 9; ++lb) {
          const int bx = lb % 3, by = lb / 3;
          const double gb0 = w[3 + bx] * w[6 + by];
          const double gb1 = w[bx] * w[9 + by];
#pragma unroll
          for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < 2; ++c)
              K[lb][r * 2 + c] = fma(U[r][c][1], gb1, fma(U[r][c][0], gb0, K[lb][r * 2 + c]));
        }
      }
#pragma unroll
      for (int lb = 0; lb < 9; ++lb)
#pragma unroll
        for (int e = 0; e < 4; ++e) part[rl][q][lb * 4 + e] = K[lb][e];
    }
  }
  __syncthreads();
  // BSR block (a, b) at stencil offset (dx, dy) = b - a: groups (qx, qy) with
  // qx in [max(0, dx), min(2, dx + 2)] (likewise y) hold both nodes; node b
  // sits at (dx + 2 - qx, dy + 2 - qy) in their stencil.  Groups off the grid
  // left zeros in LDS, so adding them changes no bit of the sum.
#pragma unroll
  for (int h = 0; h < JB; ++h) {
    if (sl[h] < 0) continue;
    const int t = threadIdx.x + 256 * h;
    const int r2 = t / 25, o = t % 25;
    const int dx = o % 5 - 2, dy = o / 5 - 2;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int qy = max(0, dy); qy <= min(2, dy + 2); ++qy)
      for (int qx = max(0, dx); qx <= min(2, dx + 2); ++qx) {
        const int qq = qy * 3 + qx;
        const int lb = (dx + 2 - qx) + 3 * (dy + 2 - qy);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] += part[r2][qq][lb * 4 + e];
      }
    if (code[h]) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          if (((code[h] >> (2 + i)) | (code[h] >> j)) & 1) acc[i * 2 + j] = (o == 12 && i == j) ? 1.0 : 0.0;
    }
    double* blk = val + ((int64_t)rp[h] + sl[h]) * 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) blk[e] = acc[e];
  }
}

// u-p Jacobian without atomics, the same two passes with 3x3 blocks.
// k_tan2up: eight lanes per particle, lane q < 7 writes column q of the 7x7
// table V0 d(P, s1, vv)/d(dF, p, grad p) (output-major), and lane 7 the
// stencil's weights and derivatives per axis.
__global__ void __launch_bounds__(256) k_tan2up(AsmArgs A, const double* __restrict__ du, double* __restrict__ pdat) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = gid >> 3;
  const int q = (int)(gid & 7);
  if (i >= A.np) return;
  PLoad<2> L;
  load_particle<2>(A, i, du, L);
  double* P = pdat + i * PU2;
  if (q < 7) {
    double Tc[7];
    tangent2_col<7>(A, L, load_be2(A, i), q, Tc);
#pragma unroll
    for (int o = 0; o < 7; ++o) P[o * 7 + q] = L.v0 * Tc[o];
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      P[49 + a] = L.st.w[0][a];
      P[52 + a] = L.st.dw[0][a];
      P[55 + a] = L.st.w[1][a];
      P[58 + a] = L.st.dw[1][a];
    }
  }
}

// k_jac2up_rows: JRU rows of 16 lanes; lane q < 9 of row a takes the q-th
// stencil group holding node a and accumulates the nine 3x3 blocks (a, b) of
// its particles, in order, in LDS.  Node a's side is contracted first: with
// (ga0, ga1) = grad w_a and wa = w_a, U[r][k] = sum over the outputs o of row
// component r (P rows for r < 2, the fluid outputs (s1, vv) for r = 2) of
// their weight times T[o][k]; then K_ab[r][c] sums U[r][k] over the inputs k
// of column component c with node b's weights (dF entries for c < 2,
// (p, grad p) for c = 2).  The block pass sums the groups holding both nodes
// in group order and writes each block once, Dirichlet from the row codes.
constexpr int JRU = 8;                          // rows per workgroup (16 lanes each)
constexpr int JBU = (JRU * 25 + JRU * 16 - 1) / (JRU * 16);   // stencil offsets per thread
__global__ void __launch_bounds__(JRU * 16) k_jac2up_rows(int64_t n_row, const int32_t* __restrict__ rgrp,
                                                         const double* __restrict__ pdat,
                                                         const int32_t* __restrict__ rowptr,
                                                         const int8_t* __restrict__ slot,
                                                         const uint8_t* __restrict__ bcode, double* __restrict__ val) {
  constexpr int NT = JRU * 16;
  __shared__ double part[JRU][9][81];   // [row][group q][local node b][3x3]
  const int rl = threadIdx.x / 16, q = threadIdx.x % 16;
  const int64_t row0 = (int64_t)blockIdx.x * JRU;
  int32_t sl[JBU], rp[JBU];
  uint32_t code[JBU];
#pragma unroll
  for (int h = 0; h < JBU; ++h) {
    const int t = threadIdx.x + NT * h;
    const int64_t row = row0 + t / 25;
    sl[h] = -1;
    rp[h] = 0;
    code[h] = 0;
    if (t < JRU * 25 && row < n_row) {
      sl[h] = slot[row * 25 + t % 25];
      rp[h] = rowptr[row];
      if (bcode) code[h] = bcode[row * 25 + t % 25];
    }
  }
  {
    const int64_t row = row0 + rl;
    if (row < n_row && q < 9) {
      const int p0 = rgrp[(row * 9 + q) * 2], p1 = rgrp[(row * 9 + q) * 2 + 1];
      const int ax = 2 - q % 3, ay = 2 - q / 3;   // node a's place in the group's 3x3 stencil
      double* K = part[rl][q];
      for (int e = 0; e < 81; ++e) K[e] = 0.0;
      for (int p = p0; p < p1; ++p) {
        const double* P = pdat + (int64_t)p * PU2;
        double w[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] = P[49 + k];
        // w: wx 0..2, dwx 3..5, wy 6..8, dwy 9..11
        const double wxa = sel3(ax, w[0], w[1], w[2]), dwxa = sel3(ax, w[3], w[4], w[5]);
        const double wya = sel3(ay, w[6], w[7], w[8]), dwya = sel3(ay, w[9], w[10], w[11]);
        const double ga0 = dwxa * wya, ga1 = wxa * dwya, wa = wxa * wya;
        double U[3][7];
#pragma unroll
        for (int k = 0; k < 7; ++k) {
          U[0][k] = fma(ga1, P[1 * 7 + k], ga0 * P[0 * 7 + k]);
          U[1][k] = fma(ga1, P[3 * 7 + k], ga0 * P[2 * 7 + k]);
          U[2][k] = fma(ga1, P[6 * 7 + k], fma(ga0, P[5 * 7 + k], wa * P[4 * 7 + k]));
        }
#pragma unroll
        for (int lb = 0; lb < 9; ++lb) {
          const int bx = lb % 3, by = lb / 3;
          const double gb0 = w[3 + bx] * w[6 + by], gb1 = w[bx] * w[9 + by], wb = w[bx] * w[6 + by];
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            double* k9 = K + lb * 9 + r * 3;
            k9[0] = fma(U[r][1], gb1, fma(U[r][0], gb0, k9[0]));
            k9[1] = fma(U[r][3], gb1, fma(U[r][2], gb0, k9[1]));
            k9[2] = fma(U[r][6], gb1, fma(U[r][5], gb0, fma(U[r][4], wb, k9[2])));
          }
        }
      }
    }
  }
  // groups off the grid (empty ranges) leave zeros; lanes of rows past the end write nothing that is read
  __syncthreads();
#pragma unroll
  for (int h = 0; h < JBU; ++h) {
    if (sl[h] < 0) continue;
    const int t = threadIdx.x + NT * h;
    const int r2 = t / 25, o = t % 25;
    const int dx = o % 5 - 2, dy = o / 5 - 2;
    double acc[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) acc[e] = 0.0;
    for (int qy = max(0, dy); qy <= min(2, dy + 2); ++qy)
      for (int qx = max(0, dx); qx <= min(2, dx + 2); ++qx) {
        const int qq = qy * 3 + qx;
        const int lb = (dx + 2 - qx) + 3 * (dy + 2 - qy);
#pragma unroll
        for (int e = 0; e < 9; ++e) acc[e] += part[r2][qq][lb * 9 + e];
      }
    if (code[h]) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          if (((code[h] >> (3 + i)) | (code[h] >> j)) & 1) acc[i * 3 + j] = (o == 12 && i == j) ? 1.0 : 0.0;
    }
    double* blk = val + ((int64_t)rp[h] + sl[h]) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) blk[e] = acc[e];
  }
}

// 32 lanes per BSR row (two rows per wave); lane k < row length owns slot k.
// With cmask, constrained rows and columns are written as the identity's.
__global__ void __launch_bounds__(256) k_jac2_blocks(int64_t n_row, const int64_t* __restrict__ active_nodes,
                                                    const int32_t* __restrict__ row_sim,
                                                    const SimDev* __restrict__ sims,
                                                    const int32_t* __restrict__ gstart,
                                                    const int32_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ colind,
                                                    const double* __restrict__ gbuf,
                                                    const uint8_t* __restrict__ cmask, double* __restrict__ val) {
  const int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 32;
  if (row >= n_row) return;
  const int k = rowptr[row] + (int)(threadIdx.x % 32);
  if (k >= rowptr[row + 1]) return;
  const SimDev& S = sims[row_sim[row]];
  const int64_t na = active_nodes[row] - S.node_base, nb = active_nodes[colind[k]] - S.node_base;
  const int ix = (int)(na % S.nna[0]) - 1, iy = (int)(na / S.nna[0]) - 1;
  const int jx = (int)(nb % S.nna[0]) - 1, jy = (int)(nb / S.nna[0]) - 1;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int oy0 = max(max(iy, jy) - 2, -1), oy1 = min(min(iy, jy), S.n[1] - 1);
  const int ox0 = max(max(ix, jx) - 2, -1), ox1 = min(min(ix, jx), S.n[0] - 1);
  for (int oy = oy0; oy <= oy1; ++oy)
    for (int ox = ox0; ox <= ox1; ++ox) {
      const int64_t key = S.okey_base + (ox + 1) + (int64_t)S.noa[0] * (oy + 1);
      if (gstart[key] == gstart[key + 1]) continue;
      const int la = (ix - ox) + 3 * (iy - oy), lb = (jx - ox) + 3 * (jy - oy);
      const double* G = gbuf + key * GB2 + (la * 9 + lb) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] += G[e];
    }
  if (cmask) {
    const int64_t col = colind[k];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        if (cmask[row * 2 + i] || cmask[col * 2 + j]) acc[i * 2 + j] = (row == col && i == j) ? 1.0 : 0.0;
  }
  double* blk = val + (int64_t)k * 4;
#pragma unroll
  for (int e = 0; e < 4; ++e) blk[e] = acc[e];
}

// 2-D residual P2G without atomics.  k_fint2_rec writes one record per
// particle (sorted order): V0 P (4), for u-p V0 s1 and V0 vv (3), then the
// stencil's weights and derivatives per axis.  k_fint2_rows gives each row
// (node a) 16 lanes: lane q < 9 sums f_a = sum_p V0 P_p grad w_a(x_p) (and the
// u-p row) over the particles of the q-th stencil group whose stencil may
// hold a (its range from the row group table), in particle order, and the 16 lane sums meet in a fixed butterfly:
// deterministic, written once.
constexpr int RD2 = 20;   // doubles per residual record: V0 P 0..3, u-p 4..6, wx 8..10, dwx 11..13, wy 14..16, dwy 17..19

__global__ void __launch_bounds__(256) k_fint2_rec(AsmArgs A, const double* __restrict__ du, double* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= A.np) return;
  PLoad<2> L;
  load_particle<2>(A, i, du, L);
  Mat<double> m = make_mat<double>(L.E, A.nu, L.phi, A.c, A.psi, A.dp, A.match, A.apex_reg);
  Out2<double> o;
  mech2<double>(m, L.dF, load_be2(A, i), L.Jn, A.up, up_par(A), L.pp, L.gp, o, nullptr);
  double* R = rec + i * RD2;
  R[0] = L.v0 * o.P[0][0]; R[1] = L.v0 * o.P[0][1];
  R[2] = L.v0 * o.P[1][0]; R[3] = L.v0 * o.P[1][1];
  R[4] = A.up ? L.v0 * o.s1 : 0.0;
  R[5] = A.up ? L.v0 * o.vv[0] : 0.0;
  R[6] = A.up ? L.v0 * o.vv[1] : 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R[8 + a] = L.st.w[0][a];
    R[11 + a] = L.st.dw[0][a];
    R[14 + a] = L.st.w[1][a];
    R[17 + a] = L.st.dw[1][a];
  }
}

constexpr int RL2 = 16;   // lanes per row of the 2-D row gathers (9 stencil groups used)

__global__ void __launch_bounds__(256, 8) k_fint2_rows(int64_t n_row, int nd, int up,
                                                   const int32_t* __restrict__ rgrp,
                                                   const double* __restrict__ rec, double* __restrict__ fint) {
  const int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) / RL2;
  const int q = (int)(threadIdx.x % RL2);
  if (row >= n_row) return;   // the row's 16 lanes leave together
  double f0 = 0.0, f1 = 0.0, f2 = 0.0;
  if (q < 9) {
    const int p0 = rgrp[(row * 9 + q) * 2], p1 = rgrp[(row * 9 + q) * 2 + 1];
    const int ax = 2 - q % 3, ay = 2 - q / 3;   // node a's place in the group's 3x3 stencil
    // the loads of two particles are issued before their sums, which take
    // the particles in order
    for (int pb = p0; pb < p1; pb += 2) {
      double v[2][8];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const double* R = rec + (int64_t)min(pb + u, p1 - 1) * RD2;
        v[u][0] = R[0]; v[u][1] = R[1]; v[u][2] = R[2]; v[u][3] = R[3];
        v[u][4] = R[8 + ax]; v[u][5] = R[11 + ax]; v[u][6] = R[14 + ay]; v[u][7] = R[17 + ay];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (pb + u >= p1) break;
        const double wx = v[u][4], dwx = v[u][5], wy = v[u][6], dwy = v[u][7];
        const double ga0 = dwx * wy, ga1 = wx * dwy;
        f0 += fma(v[u][0], ga0, v[u][1] * ga1);
        f1 += fma(v[u][2], ga0, v[u][3] * ga1);
        if (up) {
          const double* R = rec + (int64_t)(pb + u) * RD2;
          f2 += fma(wx * wy, R[4], fma(ga0, R[5], ga1 * R[6]));
        }
      }
    }
  }
#pragma unroll
  for (int off = RL2 / 2; off > 0; off >>= 1) {
    f0 += __shfl_xor(f0, off, RL2);
    f1 += __shfl_xor(f1, off, RL2);
    f2 += __shfl_xor(f2, off, RL2);
  }
  if (q == 0) {
    fint[row * nd] = f0;
    fint[row * nd + 1] = f1;
    if (up) fint[row * nd + 2] = f2;
  }
}

// ---------------------------------------------- group-cooperative 3-D ------
constexpr int GP3 = 64;   // particles (threads) per workgroup in 3-D

// 3-D Jacobian, each 3x3 block written once.
//
// k_dF3: one thread per particle gathers du over its 27 nodes once: the
// increment gradient dF [9][np] for k_tan3v, and the stencil's weights and
// derivatives per axis into the tail of the particle's tangent record
// (evaluated once here instead of at every staging below).
//
// k_tan3v: nine lanes per particle, lane q = 3c + j carrying the direction
// dF_cj, read dF and write the particle's tangent table: V0 dP_ri/dF_cj at
// [(r*3 + c)*9 + i*3 + j].
//
// k_jac3_lines: one workgroup owns a segment of JL_SEG consecutive rows of one
// x-line of nodes (fixed iy, iz) and sweeps the stencil-group origins ox along
// x.  At step ox the nine groups (ox, iy - ly, iz - lz), ly, lz in 0..2, are
// the only ones holding rows ox .. ox+2 of the line; their particles' tangent
// records (table, then the stencil's weights and derivatives per axis) are
// staged in LDS; stencil node b = (bx, by, bz) has the gradient
//   g_b = (dwx[bx] wy[by] wz[bz], wx[bx] dwy[by] wz[bz], wx[bx] wy[by] dwz[bz]),
// and a lane forms ta . g_b as (u0 wy + u1 dwy) wz + (u2 wy) dwz with
// u = (ta0 dwx, ta1 wx, ta2 wx), two FMAs per block entry,
// every (group, row, r, c) lane contracts its group's particles into the 27
// blocks of its row, the nine groups' partial blocks meet in LDS and are
// added to the rows' accumulators in a fixed group order, and row ox, which
// no later step touches, is written to its BSR row with the Dirichlet rows
// and columns applied.  So the matrix needs no clearing, no colour passes and
// no second pass for the boundary conditions, and the result does not depend
// on the launch.  A multigrid level runs the same kernel on its own grid
// over its quadrature particles' records.
// Origins of colour (cx, cy, cz) along one axis: v = o + 1 in [0, n] with v = c mod 3.
__device__ __host__ __forceinline__ int colour_count(int n, int c) { return c > n ? 0 : (n - c) / 3 + 1; }

constexpr int TL3 = 256;   // k_tan3v threads: 4 waves of 7 particles x 9 directions (63 of 64 lanes)
constexpr int TP3 = 28;    // particles per k_tan3v workgroup

__global__ void __launch_bounds__(256) k_dF3(AsmArgs A, const double* __restrict__ du, double* __restrict__ dF,
                                             double* __restrict__ rec) {
  // the stencil data pass through LDS so that the record tails leave in
  // 144-byte runs (one per particle) instead of one scattered double per lane
  __shared__ double sW[256 * 18];
  const int t = threadIdx.x;
  const int64_t p0 = (int64_t)blockIdx.x * 256, i = p0 + t;
  if (i < A.np) {
    PLoad<3> L;
    load_particle3_lean(A, i, du, L);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) dF[(r * 3 + c) * A.np + i] = L.dF[r][c];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sW[t * 18 + 6 * ax + a] = L.st.w[ax][a];
        sW[t * 18 + 6 * ax + 3 + a] = L.st.dw[ax][a];
      }
  }
  __syncthreads();
  const int n = (int)min((int64_t)256, A.np - p0);
  for (int e = t; e < n * 18; e += 256) {
    const int p = e / 18;
    rec[(p0 + p) * PTW3 + PT3 + (e - 18 * p)] = sW[e];
  }
}

__global__ void __launch_bounds__(TL3) k_tan3v(AsmArgs A, const double* __restrict__ dFs, double* __restrict__ rec,
                                               int32_t* __restrict__ flag) {
  // each lane writes its nine entries straight to the record: staging the
  // tables in LDS behind a workgroup barrier measured slower in the Newton
  // loop, where plastic returns make the waves' work uneven
  const int wl = threadIdx.x % 64;
  if (wl >= 63) return;
  const int64_t i = (int64_t)blockIdx.x * TP3 + (threadIdx.x / 64) * 7 + wl / 9;
  const int q = wl % 9;
  if (i >= A.np) return;
  const double v0 = A.vs[i], E = A.Es ? A.Es[i] : A.E, phi = A.phis ? A.phis[i] : A.phi;
  // the material constants carry no derivative here
  const Mat<double> m = make_mat<double>(E, A.nu, phi, A.c, A.psi, A.dp, A.match, A.apex_reg);
  Sym3<double> be = load_be3(A, i);
  dnum F[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) F[r][c] = dnum(dFs[(r * 3 + c) * A.np + i], q == r * 3 + c ? 1.0 : 0.0);
  Sym3<dnum> bd;
#pragma unroll
  for (int k = 0; k < 6; ++k) bd.a[k] = dnum(be.a[k]);
  Out3<dnum> o;
  int rerr = 0;
  mech3<dnum, double>(m, F, bd, o, nullptr, &rerr);
  if (rerr) atomicOr(flag, 4);
  double* R = rec + i * PTW3;
  const int c = q / 3, j = q % 3;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) R[(r * 3 + c) * 9 + ii * 3 + j] = v0 * o.P[r][ii].d;
}

constexpr int JL_T = 256;    // threads; lane t < 243 is (group q, row la_x, r, c), c fastest
constexpr int JL_SEG = 12;   // rows of a line per workgroup (cube Jacobian with its tangent records, ms:
                             // 10: 43.0, 12: 40.2, 16: 42.0, 20: 40.5, 24: 40.9; LDS strides padded
                             // against bank conflicts measured 40.9)
constexpr int JL_CH = 72;    // records staged per chunk: a step's nine groups of eight particles
constexpr int JL_BUF = JL_CH * PTW3;         // staged records (table and stencil data); then the partial blocks
constexpr int JL_PART = 6561;                 // doubles of the nine groups' partial blocks (9 x 3 rows x 27 x 9)
constexpr int JL_IT = 2;                      // accumulator blocks per thread: (slot, offset) items t, t + 256
static_assert(JL_PART <= JL_BUF, "the partial blocks reuse the staging buffer");
static_assert(JL_IT * JL_T >= 375, "every (slot, offset) item has an owner");

__device__ __forceinline__ int imod3(int v) { return ((v % 3) + 3) % 3; }

// Owned accumulator items (slot sl of the three rows in flight, offset d of
// the 5^3 neighbourhood) in an order that keeps the work of a wave uniform:
// the 25 (dy, dz) layers by the number of the nine groups that can hold both
// nodes ((3 - |dy|)(3 - |dz|): 9, then 6, 4, 3, 2, 1), 15 items (sl, dx) each.
// Thread t owns position 64 c + (t mod 64) for chunk c = t / 64 (h = 0) and
// c = 7 - t / 64 (h = 1), so the wave with the nine-group layer gets no
// second chunk.  Returns the item sl * 125 + d, or -1.
__device__ __forceinline__ int jl_item(int t, int h) {
  constexpr int8_t LDY[25] = {0, 0, 0, -1, 1, -1, -1, 1, 1, 0, 0, -2, 2, -1, -1, 1, 1, -2, -2, 2, 2, -2, -2, 2, 2};
  constexpr int8_t LDZ[25] = {0, -1, 1, 0, 0, -1, 1, -1, 1, -2, 2, 0, 0, -2, 2, -2, 2, -1, 1, -1, 1, -2, 2, -2, 2};
  const int w = t >> 6, chunk = h == 0 ? w : 7 - w;
  const int pos = chunk * 64 + (t & 63);
  if (pos >= 375) return -1;
  const int layer = pos / 15, within = pos - layer * 15;
  const int sl = within / 5, dx = within - sl * 5 - 2;
  return sl * 125 + (dx + 2) + 5 * (LDY[layer] + 2) + 25 * (LDZ[layer] + 2);
}

// Particle range [a, b) of group k of sweep step ox: origin (ox, iy - k % 3, iz - k / 3).
__device__ __forceinline__ void line_group_range(const SimDev& S, const int32_t* __restrict__ gstart, int ox, int iy,
                                                 int iz, int k, int& a, int& b) {
  const int oy = iy - (k % 3), oz = iz - (k / 3);
  a = 0;
  b = 0;
  if (oy >= -1 && oy <= S.n[1] - 1 && oz >= -1 && oz <= S.n[2] - 1) {
    const int64_t key = S.okey_base + (ox + 1) + (int64_t)S.noa[0] * ((oy + 1) + (int64_t)S.noa[1] * (oz + 1));
    a = gstart[key];
    b = gstart[key + 1];
  }
}

// The three rows in flight live in registers: thread t owns the 3x3 blocks
// of two of the 3 x 125 (slot, offset) items (slot imod3(ix) of row ix,
// offset d of the 5^3 neighbourhood; jl_item), adds the nine groups'
// partials to them in group order after every step, and writes the finished
// row's blocks itself.  Each step loads nothing that it waits for at once except
// the records it stages: the next step's group ranges and the finished row's
// slots and Dirichlet codes are loaded a step ahead, or at the step's start
// and used at its end.
__global__ void __launch_bounds__(JL_T, 2) k_jac3_lines(const int64_t* __restrict__ wstart, int nsim,
                                                        const SimDev* __restrict__ sims,
                                                        const int32_t* __restrict__ gstart,
                                                        const int32_t* __restrict__ node_map,
                                                        const double* __restrict__ rec,
                                                        const int32_t* __restrict__ pmap,
                                                        const int32_t* __restrict__ rowptr,
                                                        const int8_t* __restrict__ slot,
                                                        const uint8_t* __restrict__ bcode, double* __restrict__ val) {
  __shared__ double sbuf[JL_BUF];    // staged records [JL_CH][PTW3]; then the nine groups' partial blocks
  __shared__ int32_t rng[2][9][2];   // group ranges of this step and the next: first particle, count
  __shared__ int32_t srow[JL_SEG];
  // Workgroups are dealt to the 8 XCDs in turn; XCD x takes the x-th
  // contiguous eighth of the lines (z fastest), so lines that share stencil
  // groups run side by side on one L2.
  const unsigned nwg = gridDim.x, xcd = blockIdx.x % 8, kq = blockIdx.x / 8;
  const unsigned q8 = nwg / 8, r8 = nwg % 8;
  const int64_t w = (int64_t)xcd * q8 + min(xcd, r8) + kq;   // a bijection of [0, nwg)
  int s = 0;
  while (s + 1 < nsim && wstart[s + 1] <= w) ++s;   // workgroup-uniform
  const SimDev& S = sims[s];
  const int64_t loc = w - wstart[s];
  const int iz = (int)(loc % S.nna[2]) - 1;
  const int iy = (int)((loc / S.nna[2]) % S.nna[1]) - 1;
  const int seg = (int)(loc / ((int64_t)S.nna[2] * S.nna[1]));
  const int x0 = -1 + seg * JL_SEG;
  const int x1 = min(x0 + JL_SEG, S.n[0] + 2);   // rows x0 .. x1-1 (nodes run to n+1)
  const int t = threadIdx.x;
  const int64_t line_base = S.node_base + (int64_t)S.nna[0] * ((iy + 1) + (int64_t)S.nna[1] * (iz + 1));
  if (t < x1 - x0) srow[t] = node_map[line_base + (x0 + t + 1)];
  const int ox_lo = max(x0 - 2, -1), ox_hi = min(x1 - 1, S.n[0] - 1);
  int ra = 0, rb = 0;   // thread k < 9: range of group k, one step ahead
  if (t < 9 && ox_lo <= ox_hi) line_group_range(S, gstart, ox_lo, iy, iz, t, ra, rb);
  __syncthreads();
  {
    int any = 0;
    for (int k = 0; k < x1 - x0; ++k) any |= srow[k] >= 0;
    if (!any) return;   // no active row in this segment (uniform)
  }
  const bool lane = t < 243;
  const int c = t % 3, r = (t / 3) % 3, la_x = (t / 9) % 3, q = t / 27;
  const int ly = q % 3, lz = q / 3;   // row node's place in group q's stencil along y and z
  // owned accumulator items: slot sl, offset d
  double racc[JL_IT][9];
#pragma unroll
  for (int h = 0; h < JL_IT; ++h)
#pragma unroll
    for (int e = 0; e < 9; ++e) racc[h][e] = 0.0;

  for (int ox = ox_lo; ox <= ox_hi + 2; ++ox) {
    const int cur = ox & 1;
    if (t < 9) {
      rng[cur][t][0] = ra;
      rng[cur][t][1] = rb - ra;
      if (ox + 1 <= ox_hi) line_group_range(S, gstart, ox + 1, iy, iz, t, ra, rb);
    }
    // row ox is finished after this step: the slots and codes of its owned
    // blocks, in flight meanwhile
    const int sl0 = imod3(ox);
    const int32_t frow = (ox >= x0 && ox < x1) ? srow[ox - x0] : -1;
    int32_t fsp[JL_IT];
    uint32_t fcode[JL_IT];
    int64_t frp = 0;
#pragma unroll
    for (int h = 0; h < JL_IT; ++h) { fsp[h] = -1; fcode[h] = 0; }
    if (frow >= 0) {
      frp = rowptr[frow];
#pragma unroll
      for (int h = 0; h < JL_IT; ++h) {
        const int it = jl_item(t, h);
        if (it >= 0 && it / 125 == sl0) {
          const int d = it - sl0 * 125;
          fsp[h] = slot[(int64_t)frow * 125 + d];
          if (bcode) fcode[h] = bcode[(int64_t)frow * 125 + d];
        }
      }
    }
    __syncthreads();   // this step's ranges are visible; the last step's partials are consumed
    if (ox <= ox_hi) {
      int g0[9], goff[10];
      goff[0] = 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        g0[k] = rng[cur][k][0];
        goff[k + 1] = goff[k] + rng[cur][k][1];
      }
      const int ntot = goff[9];
      if (ntot > 0) {
        double acc[27];
#pragma unroll
        for (int b = 0; b < 27; ++b) acc[b] = 0.0;
        const int ixr = ox + la_x;
        const bool mine = lane && ixr >= x0 && ixr < x1 && srow[ixr - x0] >= 0;
        int qb = 0, qe = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k)
          if (lane && q == k) { qb = goff[k]; qe = goff[k + 1]; }
        for (int c0 = 0; c0 < ntot; c0 += JL_CH) {
          const int nc = min(JL_CH, ntot - c0);
          if (c0 > 0) __syncthreads();   // the previous chunk is consumed
          // four threads per staged particle copy its record, entries
          // part + 4 m (JL_CH * 4 > JL_T: two rounds)
          for (int u4 = t; u4 < 4 * nc; u4 += JL_T) {
            const int k = u4 >> 2, part = u4 & 3;
            const int gpos = c0 + k;
            int qq = 0;
#pragma unroll
            for (int u = 1; u < 9; ++u) qq += gpos >= goff[u];
            int gbase = g0[0], gstart_q = goff[0];
#pragma unroll
            for (int u = 1; u < 9; ++u)
              if (qq == u) { gbase = g0[u]; gstart_q = goff[u]; }
            const int64_t p = gbase + gpos - gstart_q;
            const double* src = rec + (int64_t)(pmap ? pmap[p] : p) * PTW3;
            constexpr int NM = (PTW3 + 3) / 4;   // 25: entries part + 4 m < PTW3
            double v[NM];
#pragma unroll
            for (int m = 0; m < NM; ++m) v[m] = (part + 4 * m < PTW3) ? src[part + 4 * m] : 0.0;
#pragma unroll
            for (int m = 0; m < NM; ++m)
              if (part + 4 * m < PTW3) sbuf[k * PTW3 + part + 4 * m] = v[m];
          }
          __syncthreads();
          if (mine) {
            const int kb = max(qb, c0) - c0, ke = min(qe, c0 + nc) - c0;
            for (int k = kb; k < ke; ++k) {
              const double* T = sbuf + k * PTW3 + (r * 3 + c) * 9;
              const double* R = sbuf + k * PTW3 + PT3;
              double wx[3], dwx[3], wy[3], dwy[3], wz[3], dwz[3];
#pragma unroll
              for (int u = 0; u < 3; ++u) {
                wx[u] = R[u]; dwx[u] = R[3 + u];
                wy[u] = R[6 + u]; dwy[u] = R[9 + u];
                wz[u] = R[12 + u]; dwz[u] = R[15 + u];
              }
              // node a: (la_x, ly, lz) of the group's stencil, ly = q mod 3,
              // lz = q / 3; its weights read at lane-dependent addresses
              const double wxa = R[la_x], dwxa = R[3 + la_x], wya = R[6 + ly], dwya = R[9 + ly],
                           wza = R[12 + lz], dwza = R[15 + lz];
              const double ga0 = dwxa * (wya * wza), ga1 = wxa * (dwya * wza), ga2 = wxa * (wya * dwza);
              double ta[3];
#pragma unroll
              for (int jj = 0; jj < 3; ++jj) ta[jj] = fma(ga0, T[jj], fma(ga1, T[3 + jj], ga2 * T[6 + jj]));
              double u0[3], u1[3], u2[3];
#pragma unroll
              for (int bx = 0; bx < 3; ++bx) { u0[bx] = ta[0] * dwx[bx]; u1[bx] = ta[1] * wx[bx]; u2[bx] = ta[2] * wx[bx]; }
              // ta . g_b = (u0 wy + u1 dwy) wz + (u2 wy) dwz over (bx, by), bz
#pragma unroll
              for (int by = 0; by < 3; ++by)
#pragma unroll
                for (int bx = 0; bx < 3; ++bx) {
                  const double X = fma(u1[bx], dwy[by], u0[bx] * wy[by]), Y = u2[bx] * wy[by];
#pragma unroll
                  for (int bz = 0; bz < 3; ++bz) {
                    const int b = bx + 3 * by + 9 * bz;
                    acc[b] = fma(X, wz[bz], fma(Y, dwz[bz], acc[b]));
                  }
                }
            }
          }
        }
        __syncthreads();   // the staged records are consumed
        if (lane) {
#pragma unroll
          for (int b = 0; b < 27; ++b) sbuf[((q * 3 + la_x) * 27 + b) * 9 + r * 3 + c] = mine ? acc[b] : 0.0;
        }
        __syncthreads();
        // owned items add the nine groups' partials in group order, visiting
        // only the groups that hold both nodes (the same count across most
        // of a wave, by the item order)
#pragma unroll
        for (int h = 0; h < JL_IT; ++h) {
          const int it = jl_item(t, h);
          if (it < 0) continue;
          const int sl = it / 125, d = it - sl * 125;
          const int lx = imod3(sl - ox);   // row ox + lx sits in slot sl
          const int dx = d % 5 - 2, dy = (d / 5) % 5 - 2, dz = d / 25 - 2;
          const int bx = lx + dx;
          if (bx < 0 || bx > 2) continue;
          double sum[9];
#pragma unroll
          for (int e = 0; e < 9; ++e) sum[e] = 0.0;
          const int qy0 = max(0, -dy), qy1 = min(2, 2 - dy), qz0 = max(0, -dz), qz1 = min(2, 2 - dz);
          for (int qz = qz0; qz <= qz1; ++qz)
            for (int qy = qy0; qy <= qy1; ++qy) {
              const int qq = qy + 3 * qz;
              const double* src = sbuf + ((qq * 3 + lx) * 27 + bx + 3 * (qy + dy) + 9 * (qz + dz)) * 9;
#pragma unroll
              for (int e = 0; e < 9; ++e) sum[e] += src[e];
            }
#pragma unroll
          for (int e = 0; e < 9; ++e) racc[h][e] += sum[e];
        }
      }
    }
    // row ox is finished (the last two steps only flush): write its owned
    // blocks, clear them
    if (ox >= x0 && ox < x1) {
#pragma unroll
      for (int h = 0; h < JL_IT; ++h) {
        const int it = jl_item(t, h);
        if (it < 0 || it / 125 != sl0) continue;
        const int d = it - sl0 * 125;
        if (frow >= 0 && fsp[h] >= 0) {
          double* blk = val + (frp + fsp[h]) * 9;
#pragma unroll
          for (int rc = 0; rc < 9; ++rc) {
            double out = racc[h][rc];
            const int rr = rc / 3, cc = rc - rr * 3;
            if (((fcode[h] >> (3 + rr)) | (fcode[h] >> cc)) & 1u) out = (d == 62 && rr == cc) ? 1.0 : 0.0;
            blk[rc] = out;
          }
        }
#pragma unroll
        for (int e = 0; e < 9; ++e) racc[h][e] = 0.0;
      }
    }
  }
}

// 3-D external force without atomics: per particle a force record (the
// particle's force and its stencil weights and derivatives, written by the
// pattern build), then k_p2g3c gives one workgroup to each stencil group of a
// colour and adds the group's sum over its particles, in order, to each of
// its 27 nodes with a plain read-modify-write.
constexpr int PR3 = 28;    // doubles per 3-D force record: V0 P 0..8 (or the force 0..2), w 9..17 [axis][a], dw 18..26

// mode 0: f_a += sum_p V0 P_p grad w_a(x_p) (internal force);
// mode 1: f_a += sum_p w_a(x_p) f_p (external force).
constexpr int PG3 = 32;   // records staged in LDS at a time
__global__ void __launch_bounds__(64) k_p2g3c(int colour, int mode, const int64_t* __restrict__ wstart, int nsim,
                                             const SimDev* __restrict__ sims, const int32_t* __restrict__ gstart,
                                             const int32_t* __restrict__ node_map, const double* __restrict__ rec,
                                             double* __restrict__ out) {
  __shared__ double sR[PG3][PR3];
  const int64_t w = blockIdx.x;
  int s = 0;
  while (s + 1 < nsim && wstart[s + 1] <= w) ++s;   // workgroup-uniform
  const SimDev& S = sims[s];
  const int cx = colour % 3, cy = (colour / 3) % 3, cz = colour / 9;
  const int nx = colour_count(S.n[0], cx), ny = colour_count(S.n[1], cy);
  const int64_t loc = w - wstart[s];
  const int ox = cx + 3 * (int)(loc % nx) - 1, oy = cy + 3 * (int)((loc / nx) % ny) - 1,
            oz = cz + 3 * (int)(loc / ((int64_t)nx * ny)) - 1;
  const int64_t key = S.okey_base + (ox + 1) + (int64_t)S.noa[0] * ((oy + 1) + (int64_t)S.noa[1] * (oz + 1));
  const int p0 = gstart[key], p1 = gstart[key + 1];
  if (p0 == p1) return;   // empty origin (uniform over the workgroup)
  const int t = threadIdx.x;
  const int ax = t % 3, ay = (t / 3) % 3, az = t / 9;
  double f0 = 0.0, f1 = 0.0, f2 = 0.0;
  for (int c0 = p0; c0 < p1; c0 += PG3) {
    const int nc = min(PG3, p1 - c0);
    __syncthreads();   // the previous chunk is consumed
    for (int e = t; e < nc * PR3; e += 64) sR[e / PR3][e % PR3] = rec[(int64_t)c0 * PR3 + e];
    __syncthreads();
    if (t < 27) {
      for (int p = 0; p < nc; ++p) {
        const double* R = sR[p];
        if (mode == 0) {
          const double ga0 = R[18 + ax] * R[12 + ay] * R[15 + az];
          const double ga1 = R[9 + ax] * R[21 + ay] * R[15 + az];
          const double ga2 = R[9 + ax] * R[12 + ay] * R[24 + az];
          f0 += R[0] * ga0 + R[1] * ga1 + R[2] * ga2;
          f1 += R[3] * ga0 + R[4] * ga1 + R[5] * ga2;
          f2 += R[6] * ga0 + R[7] * ga1 + R[8] * ga2;
        } else {
          const double wa = R[9 + ax] * R[12 + ay] * R[15 + az];
          f0 += wa * R[0];
          f1 += wa * R[1];
          f2 += wa * R[2];
        }
      }
    }
  }
  if (t < 27) {
    const int32_t ra = node_map[S.node_base + (ox + ax + 1) + (int64_t)S.nna[0] * ((oy + ay + 1) + (int64_t)S.nna[1] * (oz + az + 1))];
    double* f = out + (int64_t)ra * 3;
    f[0] += f0;   // one writer per node in this colour
    f[1] += f1;
    f[2] += f2;
  }
}

// 3-D internal force in one pass per colour, without particle records:
// a workgroup takes FG3 consecutive stencil groups of one colour (no two of
// them share a node), evaluates their particles' stresses into LDS (64 at a
// time) and then adds each group's sum over its particles, in order, to each
// of the group's 27 nodes with a plain read-modify-write.  Every particle is
// evaluated once, and f_int is deterministic.
constexpr int FG3 = 7;    // stencil groups per workgroup (seven: one scatter task (group, x-node, y-node) per thread)
constexpr int FT3 = 64;   // threads (particles evaluated at a time)

// The FG3 consecutive stencil groups (of one colour) that workgroup wl of a
// sim takes: lane k < FG3 looks up group k's particle range, all lookups in
// flight at once, then lane 0 forms the offsets goff (goff[FG3]: the
// workgroup's particle count).  Groups past the colour's count are empty.
// Ends with the workgroup synchronised.
__device__ __forceinline__ void fg3_groups(const SimDev& S, const int32_t* __restrict__ gstart, int64_t wl,
                                           int colour, int t, int32_t* gp0, int32_t* gcn, int32_t* goff,
                                           int32_t* gox, int32_t* goy, int32_t* goz) {
  const int cx = colour % 3, cy = (colour / 3) % 3, cz = colour / 9;
  const int nx = colour_count(S.n[0], cx), ny = colour_count(S.n[1], cy), nz = colour_count(S.n[2], cz);
  const int64_t ngr = (int64_t)nx * ny * nz;
  if (t < FG3) {
    const int64_t g = wl * FG3 + t;
    int a = 0, b = 0, ox = 0, oy = 0, oz = 0;
    if (g < ngr) {
      ox = cx + 3 * (int)(g % nx) - 1;
      oy = cy + 3 * (int)((g / nx) % ny) - 1;
      oz = cz + 3 * (int)(g / ((int64_t)nx * ny)) - 1;
      const int64_t key = S.okey_base + (ox + 1) + (int64_t)S.noa[0] * ((oy + 1) + (int64_t)S.noa[1] * (oz + 1));
      a = gstart[key];
      b = gstart[key + 1];
    }
    gp0[t] = a; gcn[t] = b - a;
    gox[t] = ox; goy[t] = oy; goz[t] = oz;
  }
  __syncthreads();
  if (t == 0) {
    int acc = 0;
#pragma unroll
    for (int k = 0; k < FG3; ++k) { goff[k] = acc; acc += gcn[k]; }
    goff[FG3] = acc;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(FT3) __attribute__((amdgpu_waves_per_eu(2))) k_fint3c(AsmArgs A, const double* __restrict__ du, int colour,
                                                const int64_t* __restrict__ wstart, const int32_t* __restrict__ gstart,
                                                double* __restrict__ fint, int32_t* __restrict__ flag) {
  __shared__ double sP[FT3][9];              // V0 P of the staged particles
  __shared__ double sW[FT3][3][2][3];        // per axis: weights, derivatives
  __shared__ double sF[FG3 * 27][3];         // per (group, stencil node) task: its force so far
  __shared__ int32_t gp0[FG3], gcn[FG3], goff[FG3 + 1];
  __shared__ int32_t gox[FG3], goy[FG3], goz[FG3];
  const int64_t w = blockIdx.x;
  int s = 0;
  while (s + 1 < A.nsim && wstart[s + 1] <= w) ++s;   // workgroup-uniform
  const SimDev& S = A.sims[s];
  const int t = threadIdx.x;
  fg3_groups(S, gstart, w - wstart[s], colour, t, gp0, gcn, goff, gox, goy, goz);
  const int ntot = goff[FG3];
  if (ntot == 0) return;   // uniform
  // scatter tasks: (group k, stencil x-node ax, y-node ay), FG3 * 9 of them,
  // one per thread; each sums its three z-nodes with the weights factored as
  //   P grad w_a = (P0 dwx wy + P1 wx dwy) wz + (P2 wx wy) dwz,
  // and keeps the sums in LDS between chunks (no registers held across the
  // stress evaluation)
  static_assert(FG3 * 9 <= FT3, "one scatter task per thread");
  constexpr int NTK = (FG3 * 27 + FT3 - 1) / FT3;   // (group, node) items per thread in the final write
  // the rows of this thread's final-write items, fetched now so that their
  // latency hides behind the stress evaluation (-1: no item)
  int32_t rw[NTK];
#pragma unroll
  for (int j = 0; j < NTK; ++j) {
    const int tk = t + FT3 * j;
    rw[j] = -1;
    if (tk < FG3 * 27) {
      const int k = tk / 27, a = tk % 27;
      if (goff[k + 1] != goff[k]) {   // an empty group's nodes may be inactive
        const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
        rw[j] = A.node_map[S.node_base + (gox[k] + ax + 1) +
                           (int64_t)S.nna[0] * ((goy[k] + ay + 1) + (int64_t)S.nna[1] * (goz[k] + az + 1))];
      }
    }
  }
  for (int e = t; e < FG3 * 27 * 3; e += FT3) (&sF[0][0])[e] = 0.0;
  int rerr = 0;
  for (int c0 = 0; c0 < ntot; c0 += FT3) {
    const int nc = min(FT3, ntot - c0);
    if (t < nc) {
      const int gpos = c0 + t;
      int k = 0;
#pragma unroll
      for (int u = 1; u < FG3; ++u) k += gpos >= goff[u];
      const int64_t i = gp0[k] + (gpos - goff[k]);
      PLoad<3> L;
      load_particle3_lean(A, i, du, L);
      Mat<double> m = make_mat<double>(L.E, A.nu, L.phi, A.c, A.psi, A.dp, A.match, A.apex_reg);
      Out3<double> o;
      mech3<double>(m, L.dF, load_be3(A, i), o, nullptr, &rerr);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) sP[t][r * 3 + cc] = L.v0 * o.P[r][cc];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
#pragma unroll
        for (int a = 0; a < 3; ++a) { sW[t][ax][0][a] = L.st.w[ax][a]; sW[t][ax][1][a] = L.st.dw[ax][a]; }
    }
    __syncthreads();
    if (t < FG3 * 9) {
      const int k = t / 9, axy = t - 9 * k, ax = axy % 3, ay = axy / 3;
      const int kb = max(goff[k], c0) - c0, ke = min(goff[k + 1], c0 + nc) - c0;
      if (kb < ke) {
        double f[3][3];   // [az][component]
#pragma unroll
        for (int az = 0; az < 3; ++az)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) f[az][cc] = sF[k * 27 + ax + 3 * ay + 9 * az][cc];
        for (int p = kb; p < ke; ++p) {
          const double wxy0 = sW[p][0][1][ax] * sW[p][1][0][ay], wxy1 = sW[p][0][0][ax] * sW[p][1][1][ay],
                       wxy2 = sW[p][0][0][ax] * sW[p][1][0][ay];
          const double* P = sP[p];
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            const double X = fma(P[3 * cc + 1], wxy1, P[3 * cc] * wxy0), Y = P[3 * cc + 2] * wxy2;
#pragma unroll
            for (int az = 0; az < 3; ++az) f[az][cc] = fma(X, sW[p][2][0][az], fma(Y, sW[p][2][1][az], f[az][cc]));
          }
        }
#pragma unroll
        for (int az = 0; az < 3; ++az)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) sF[k * 27 + ax + 3 * ay + 9 * az][cc] = f[az][cc];   // this thread's alone
      }
    }
    __syncthreads();   // the staged particles are consumed
  }
  if (rerr) atomicOr(flag, 4);
#pragma unroll
  for (int j = 0; j < NTK; ++j) {
    if (rw[j] < 0) continue;
    const int tk = t + FT3 * j;
    double* fo = fint + (int64_t)rw[j] * 3;
    fo[0] += sF[tk][0];   // one writer per node in this colour
    fo[1] += sF[tk][1];
    fo[2] += sF[tk][2];
  }
}

// Matrix-free Jacobian-vector product (the matrix-free Newton-Krylov variant
// of Sec. 2.2, Remark 2): y = J x from the per-particle tangent records
// (V0 dP/dF) without forming the BSR matrix.  Per particle the increment
// gradient dF = sum_b x_b (x) grad w_b, the stress increment dP = T : dF,
// then dP grad w_a scattered like the internal force.  Constrained unknowns
// of x are read as zero when cm is given (the Dirichlet-modified matrix).
//
// 3-D: per colour, FG3 stencil groups per workgroup as in k_fint3c.
__global__ void __launch_bounds__(FT3) k_jv3c(int colour, const int64_t* __restrict__ wstart, int nsim,
                                              const SimDev* __restrict__ sims, const int32_t* __restrict__ gstart,
                                              const int32_t* __restrict__ node_map, const double* __restrict__ xs,
                                              int64_t np, const double* __restrict__ rec,
                                              const uint8_t* __restrict__ cm, const double* __restrict__ x,
                                              double* __restrict__ y) {
  __shared__ double sP[FT3][9];
  __shared__ double sW[FT3][3][2][3];
  __shared__ double sF[FG3 * 27][3];         // per (group, stencil node) task: its sum so far
  __shared__ int32_t gp0[FG3], gcn[FG3], goff[FG3 + 1];
  __shared__ int32_t gox[FG3], goy[FG3], goz[FG3];
  const int64_t w = blockIdx.x;
  int s = 0;
  while (s + 1 < nsim && wstart[s + 1] <= w) ++s;   // workgroup-uniform
  const SimDev& S = sims[s];
  const int t = threadIdx.x;
  fg3_groups(S, gstart, w - wstart[s], colour, t, gp0, gcn, goff, gox, goy, goz);
  const int ntot = goff[FG3];
  if (ntot == 0) return;   // uniform
  // the scatter as in k_fint3c: one task (group, x-node, y-node) per thread
  // summing its three z-nodes with factored weights, sums in LDS, and the
  // rows of the final writes fetched before the first chunk
  static_assert(FG3 * 9 <= FT3, "one scatter task per thread");
  constexpr int NTK = (FG3 * 27 + FT3 - 1) / FT3;
  int32_t rw[NTK];
#pragma unroll
  for (int j = 0; j < NTK; ++j) {
    const int tk = t + FT3 * j;
    rw[j] = -1;
    if (tk < FG3 * 27) {
      const int k = tk / 27, a = tk % 27;
      if (goff[k + 1] != goff[k]) {   // an empty group's nodes may be inactive
        const int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
        rw[j] = node_map[S.node_base + (gox[k] + ax + 1) +
                         (int64_t)S.nna[0] * ((goy[k] + ay + 1) + (int64_t)S.nna[1] * (goz[k] + az + 1))];
      }
    }
  }
  for (int e = t; e < FG3 * 27 * 3; e += FT3) (&sF[0][0])[e] = 0.0;
  for (int c0 = 0; c0 < ntot; c0 += FT3) {
    const int nc = min(FT3, ntot - c0);
    if (t < nc) {
      const int gpos = c0 + t;
      int k = 0;
#pragma unroll
      for (int u = 1; u < FG3; ++u) k += gpos >= goff[u];
      const int64_t i = gp0[k] + (gpos - goff[k]);
      Stencil<3> st;
      make_stencil<3>(S, xs, np, i, st);
      double dF[3][3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) dF[r][c] = 0.0;
#pragma unroll
      for (int az = 0; az < 3; ++az) {
        int32_t rr[9];
#pragma unroll
        for (int a9 = 0; a9 < 9; ++a9) rr[a9] = node_map[st.node(S, a9 + 9 * az)];
#pragma unroll
        for (int a9 = 0; a9 < 9; ++a9) {
          double g[3];
          st.grad(a9 + 9 * az, g);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const int64_t e = (int64_t)rr[a9] * 3 + c;
            const double xv = (cm && cm[e]) ? 0.0 : x[e];
#pragma unroll
            for (int j = 0; j < 3; ++j) dF[c][j] += xv * g[j];
          }
        }
      }
      const double* T = rec + i * PTW3;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int ii = 0; ii < 3; ++ii) {
          double a = 0.0;
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int j = 0; j < 3; ++j) a += T[(r * 3 + c) * 9 + ii * 3 + j] * dF[c][j];
          sP[t][r * 3 + ii] = a;
        }
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
#pragma unroll
        for (int a = 0; a < 3; ++a) { sW[t][ax][0][a] = st.w[ax][a]; sW[t][ax][1][a] = st.dw[ax][a]; }
    }
    __syncthreads();
    if (t < FG3 * 9) {
      const int k = t / 9, axy = t - 9 * k, ax = axy % 3, ay = axy / 3;
      const int kb = max(goff[k], c0) - c0, ke = min(goff[k + 1], c0 + nc) - c0;
      if (kb < ke) {
        double f[3][3];   // [az][component]
#pragma unroll
        for (int az = 0; az < 3; ++az)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) f[az][cc] = sF[k * 27 + ax + 3 * ay + 9 * az][cc];
        for (int p = kb; p < ke; ++p) {
          const double wxy0 = sW[p][0][1][ax] * sW[p][1][0][ay], wxy1 = sW[p][0][0][ax] * sW[p][1][1][ay],
                       wxy2 = sW[p][0][0][ax] * sW[p][1][0][ay];
          const double* P = sP[p];
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            const double X = fma(P[3 * cc + 1], wxy1, P[3 * cc] * wxy0), Y = P[3 * cc + 2] * wxy2;
#pragma unroll
            for (int az = 0; az < 3; ++az) f[az][cc] = fma(X, sW[p][2][0][az], fma(Y, sW[p][2][1][az], f[az][cc]));
          }
        }
#pragma unroll
        for (int az = 0; az < 3; ++az)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) sF[k * 27 + ax + 3 * ay + 9 * az][cc] = f[az][cc];   // this thread's alone
      }
    }
    __syncthreads();   // the staged particles are consumed
  }
#pragma unroll
  for (int j = 0; j < NTK; ++j) {
    if (rw[j] < 0) continue;
    const int tk = t + FT3 * j;
    double* yo = y + (int64_t)rw[j] * 3;
    yo[0] += sF[tk][0];   // one writer per node in this colour
    yo[1] += sF[tk][1];
    yo[2] += sF[tk][2];
  }
}

// 2-D: per particle the stress increment dP = T : dF from its tangent record
// (k_tan2 layout), written as a residual record (k_fint2_rec layout) so the
// row gather of the internal force forms y.
__global__ void __launch_bounds__(256) k_jv2_rec(int64_t np, const SimDev* __restrict__ sims,
                                                 const int32_t* __restrict__ psim, const int32_t* __restrict__ node_map,
                                                 const double* __restrict__ pdat, const uint8_t* __restrict__ cm,
                                                 const double* __restrict__ xs, const double* __restrict__ x,
                                                 double* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  const SimDev& S = sims[psim[i]];
  const double* P = pdat + i * PD2;
  const double u0 = (xs[i] - S.x0[0]) / S.h, u1 = (xs[np + i] - S.x0[1]) / S.h;
  const int o0 = (int)floor(u0 - 0.5), o1 = (int)floor(u1 - 0.5);
  double dF[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
  for (int b = 0; b < 9; ++b) {
    const int bx = b % 3, by = b / 3;
    const int32_t r = node_map[S.node_base + (o0 + bx + 1) + (int64_t)S.nna[0] * (o1 + by + 1)];
    const double g0 = P[19 + bx] * P[22 + by], g1 = P[16 + bx] * P[25 + by];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int64_t e = (int64_t)r * 2 + c;
      const double xv = (cm && cm[e]) ? 0.0 : x[e];
      dF[c][0] += xv * g0;
      dF[c][1] += xv * g1;
    }
  }
  double* R = rec + i * RD2;
#pragma unroll
  for (int o = 0; o < 4; ++o)
    R[o] = P[o * 4 + 0] * dF[0][0] + P[o * 4 + 1] * dF[0][1] + P[o * 4 + 2] * dF[1][0] + P[o * 4 + 3] * dF[1][1];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R[8 + a] = P[16 + a];
    R[11 + a] = P[19 + a];
    R[14 + a] = P[22 + a];
    R[17 + a] = P[25 + a];
  }
}

// Dirichlet rows of J_mod x: y = x on constrained unknowns.
__global__ void k_jv_bc(int64_t nv, const uint8_t* __restrict__ cm, const double* __restrict__ x,
                        double* __restrict__ y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nv && cm[e]) y[e] = x[e];
}


// ------------------------------------------------------------- update ------
template <int DIM>
__global__ void __launch_bounds__(256) k_update(AsmArgs A, const double* __restrict__ du, const int32_t* __restrict__ perm,
                         double* __restrict__ x_out, double* __restrict__ F_out, double* __restrict__ be_out,
                         int32_t* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.np) return;
  PLoad<DIM> L;
  load_particle<DIM>(A, i, du, L);
  Mat<double> m = make_mat<double>(L.E, A.nu, L.phi, A.c, A.psi, A.dp, A.match, A.apex_reg);
  const int64_t np = A.np, p = perm[i];
  const SimDev& S = A.sims[A.psim[i]];
  (void)S;
  // x^{n+1} = x^n + sum_a w_a du_a
  double dx[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) dx[k] = 0.0;
  for (int a = 0; a < Stencil<DIM>::NN; ++a) {
    double w = L.st.weight(a);
    const double* u = du + (int64_t)L.row[a] * A.nd;
#pragma unroll
    for (int k = 0; k < DIM; ++k) dx[k] += w * u[k];
  }
  double xn[DIM], Fn[DIM * DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) xn[k] = A.xs[k * np + i] + dx[k];
#pragma unroll
  for (int r = 0; r < DIM; ++r)
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) s += L.dF[r][k] * A.Fs[(k * DIM + c) * np + i];
      Fn[r * DIM + c] = s;
    }
  if constexpr (DIM == 2) {
    Out2<double> o;
    Sym2<double> b;
    double F[2][2] = {{L.dF[0][0], L.dF[0][1]}, {L.dF[1][0], L.dF[1][1]}};
    double gp0[2] = {0.0, 0.0};
    mech2<double>(m, F, load_be2(A, i), L.Jn, 0, up_par(A), 0.0, gp0, o, &b);
    if (be_out) {
      be_out[0 * np + p] = b.xx; be_out[1 * np + p] = b.yy; be_out[2 * np + p] = b.xy; be_out[3 * np + p] = b.zz;
    }
  } else {
    Out3<double> o;
    Sym3<double> b;
    int rerr = 0;
    mech3<double>(m, L.dF, load_be3(A, i), o, &b, &rerr);
    if (rerr) atomicOr(flag, 4);
    if (be_out)
#pragma unroll
      for (int t = 0; t < 6; ++t) be_out[t * np + p] = b.a[t];
  }
  if (x_out)
#pragma unroll
    for (int k = 0; k < DIM; ++k) x_out[k * np + p] = xn[k];
  if (F_out)
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) F_out[k * np + p] = Fn[k];
}

}  // namespace mpm

using namespace mpm;

// ---------------------------------------------------------------- host -----
static AsmArgs make_args(mpm_ctx* c, const mpm_problem* pb) {
  AsmArgs A;
  A.np = c->np;
  A.nsim = c->nsim;
  A.nd = c->nd;
  A.up = c->up;
  A.dp = c->dp;
  A.match = pb->mat.dp_match;
  A.xs = c->xs.p; A.vs = c->vol0s.p; A.Fs = c->Fs.p; A.bes = c->bes.p;
  A.Es = pb->P.E ? c->Es.p : nullptr;
  A.phis = pb->P.phi ? c->phis.p : nullptr;
  A.psim = c->psim.p;
  A.sims = c->sims.p;
  A.node_map = c->node_map.p;
  A.E = pb->mat.E; A.nu = pb->mat.nu; A.phi = pb->mat.phi; A.c = pb->mat.c; A.psi = pb->mat.psi;
  A.apex_reg = pb->mat.apex_reg;
  A.biot = pb->mat.biot;
  A.mob = pb->mat.mu_f > 0 ? pb->mat.perm / pb->mat.mu_f : 0.0;
  A.dt = pb->mat.dt; A.rho_f = pb->mat.rho_f;
  for (int k = 0; k < 3; ++k) A.g[k] = pb->mat.g[k];
  return A;
}

static unsigned nb256(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

// f_int into c->fint (zeroed first).
// Per colour of 3-D stencil groups and per sim, the first workgroup of the
// colour passes (groups of one colour share no node).  Built by prepare.
int build_colour_table(mpm_ctx* c) {
  const int nsim = c->nsim;
  c->jc3_ws_h.assign(27 * (size_t)(nsim + 1), 0);
  for (int col = 0; col < 27; ++col) {
    int64_t* ws = &c->jc3_ws_h[(size_t)col * (nsim + 1)];
    for (int s = 0; s < nsim; ++s) {
      const SimDev& S = c->sims_h[s];
      ws[s + 1] = ws[s] + (int64_t)colour_count(S.n[0], col % 3) * colour_count(S.n[1], (col / 3) % 3) *
                              colour_count(S.n[2], col / 9);
    }
  }
  if (c->jc3_ws.ensure(c->jc3_ws_h.size()) != hipSuccess) return c->fail(MPM_E_NOMEM, "colour table allocation failed");
  HIPC(c, hipMemcpyAsync(c->jc3_ws.p, c->jc3_ws_h.data(), c->jc3_ws_h.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                         c->stream));
  // per colour and sim the first workgroup of the fused 3-D internal force (FG3 groups each)
  c->jf3_ws_h.assign(27 * (size_t)(nsim + 1), 0);
  for (int col = 0; col < 27; ++col) {
    int64_t* ws = &c->jf3_ws_h[(size_t)col * (nsim + 1)];
    for (int s = 0; s < nsim; ++s) {
      const SimDev& S = c->sims_h[s];
      const int64_t ng = (int64_t)colour_count(S.n[0], col % 3) * colour_count(S.n[1], (col / 3) % 3) *
                         colour_count(S.n[2], col / 9);
      ws[s + 1] = ws[s] + (ng + FG3 - 1) / FG3;
    }
  }
  if (c->jf3_ws.ensure(c->jf3_ws_h.size()) != hipSuccess) return c->fail(MPM_E_NOMEM, "colour table allocation failed");
  HIPC(c, hipMemcpyAsync(c->jf3_ws.p, c->jf3_ws_h.data(), c->jf3_ws_h.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                         c->stream));
  // per sim the first workgroup of the 3-D line sweep: (n+3)^2 lines of ceil((n+3)/JL_SEG) segments
  c->jl3_ws_h.assign(nsim + 1, 0);
  for (int s = 0; s < nsim; ++s) {
    const SimDev& S = c->sims_h[s];
    c->jl3_ws_h[s + 1] = c->jl3_ws_h[s] + (int64_t)((S.nna[0] + JL_SEG - 1) / JL_SEG) * S.nna[1] * S.nna[2];
  }
  if (c->jl3_ws.ensure(nsim + 1) != hipSuccess) return c->fail(MPM_E_NOMEM, "line table allocation failed");
  HIPC(c, hipMemcpyAsync(c->jl3_ws.p, c->jl3_ws_h.data(), (nsim + 1) * sizeof(int64_t), hipMemcpyHostToDevice,
                         c->stream));
  return MPM_OK;
}

// out[row * 3 + k] += the 3-D P2G of the force records rec (mode 0 internal,
// 1 external), colour by colour.
int launch_p2g3(mpm_ctx* c, int mode, const double* rec, double* out) {
  const int nsim = c->nsim;
  for (int col = 0; col < 27; ++col) {
    const int64_t nwg = c->jc3_ws_h[(size_t)col * (nsim + 1) + nsim];
    if (nwg == 0) continue;
    k_p2g3c<<<(unsigned)nwg, 64, 0, c->stream>>>(col, mode, c->jc3_ws.p + (size_t)col * (nsim + 1), nsim, c->sims.p,
                                                 c->gstart.p, c->node_map.p, rec, out);
    LAUNCH_CHECK(c, "k_p2g3c");
  }
  return MPM_OK;
}

// Doubles per particle of the residual's force records.
int64_t fint_record_doubles(int dim) { return dim == 2 ? RD2 : 0; }

// f_int into c->fint.  rec: the force records (np * fint_record_doubles
// doubles); null uses the context's own buffer (allocated on first use).
int launch_fint(mpm_ctx* c, const mpm_problem* pb, const double* du, double* rec) {
  AsmArgs A = make_args(c, pb);
  if (!rec) {
    if (c->rrec.ensure(std::max<int64_t>(1, c->np) * fint_record_doubles(c->dim)) != hipSuccess)
      return c->fail(MPM_E_NOMEM, "residual records allocation failed");
    rec = c->rrec.p;
  }
  if (c->dim == 2) {
    // particle records, then one writer per row (deterministic, no clearing)
    if (c->np > 0) {
      k_fint2_rec<<<(unsigned)((c->np + 255) / 256), 256, 0, c->stream>>>(A, du, rec);
      LAUNCH_CHECK(c, "k_fint2_rec");
    }
    if (c->n_row > 0) {
      k_fint2_rows<<<(unsigned)((c->n_row * RL2 + 255) / 256), 256, 0, c->stream>>>(
          c->n_row, c->nd, c->up, c->rgrp.p, rec, c->fint.p);
      LAUNCH_CHECK(c, "k_fint2_rows");
    }
    return MPM_OK;
  }
  HIPC(c, hipMemsetAsync(c->fint.p, 0, c->n_row * c->nd * sizeof(double), c->stream));
  if (c->np == 0) return MPM_OK;
  // the 27 colours of stencil groups in order, stresses evaluated in place (no records)
  const int nsim = c->nsim;
  for (int col = 0; col < 27; ++col) {
    const int64_t nwg = c->jf3_ws_h[(size_t)col * (nsim + 1) + nsim];
    if (nwg == 0) continue;
    k_fint3c<<<(unsigned)nwg, FT3, 0, c->stream>>>(A, du, col, c->jf3_ws.p + (size_t)col * (nsim + 1), c->gstart.p,
                                                    c->fint.p, c->flag.p);
    LAUNCH_CHECK(c, "k_fint3c");
  }
  return MPM_OK;
}

// Residual with per-sim ||r||^2 -> simsc[s*16+0], reaction -> simsc[s*16+1].
int launch_residual(mpm_ctx* c, const mpm_problem* pb, const double* du, double* r, double* r_raw, double* rec) {
  int rc = launch_fint(c, pb, du, rec);
  if (rc) return rc;
  unsigned nbk = (unsigned)c->blocks_h.size();
  if (nbk) {
    k_res_final<<<nbk, 64, 0, c->stream>>>(c->blocks.p, c->nd, c->fint.p, c->fext.p, c->cmask.p, c->rmask.p, r, r_raw,
                                            c->part.p);
    LAUNCH_CHECK(c, "k_res_final");
  } else {
    HIPC(c, hipMemsetAsync(c->part.p, 0, NQ * sizeof(double), c->stream));
  }
  k_sim_sum_res<<<c->nsim, 64, 0, c->stream>>>(c->blk_first.p, c->part.p, c->simsc.p);
  LAUNCH_CHECK(c, "k_sim_sum_res");
  return MPM_OK;
}

int sim_sum_launch(mpm_ctx* c, const double* part, int q, int off) {
  k_sim_sum<<<c->nsim, 64, 0, c->stream>>>(c->nsim, c->blk_first.p, part, q, c->simsc.p, 16, off);
  LAUNCH_CHECK(c, "k_sim_sum");
  return MPM_OK;
}

// BSR blocks from the particle records already in c->pdat (2-D
// single-phase); apply_bc writes constrained rows and columns as the
// identity's.
int launch_jac2_records(mpm_ctx* c, double* val, bool apply_bc) {
  if (c->n_row > 0) {
    k_jac2_rows<<<(unsigned)((c->n_row + JR - 1) / JR), 256, 0, c->stream>>>(
        c->n_row, c->rgrp.p, c->pdat.p, c->rowptr.p, c->slot.p, apply_bc ? c->bcode.p : nullptr, val);
    LAUNCH_CHECK(c, "k_jac2_rows");
  }
  return MPM_OK;
}

// u-p BSR blocks of context c from its u-p records rec (c's sorted order).
int launch_jac2up_records(mpm_ctx* c, const double* rec, double* val, bool apply_bc, const int32_t* rgrp) {
  if (c->n_row > 0) {
    k_jac2up_rows<<<(unsigned)((c->n_row + JRU - 1) / JRU), JRU * 16, 0, c->stream>>>(
        c->n_row, rgrp ? rgrp : c->rgrp.p, rec, c->rowptr.p, c->slot.p, apply_bc ? c->bcode.p : nullptr, val);
    LAUNCH_CHECK(c, "k_jac2up_rows");
  }
  return MPM_OK;
}

// BSR blocks from the group blocks already in c->gbuf.
int launch_jac2_blocks(mpm_ctx* c, double* val, bool apply_bc) {
  if (c->n_row > 0) {
    k_jac2_blocks<<<(unsigned)((c->n_row * 32 + 255) / 256), 256, 0, c->stream>>>(
        c->n_row, c->active_nodes.p, c->row_sim.p, c->sims.p, c->gstart.p, c->rowptr.p, c->colind.p, c->gbuf.p,
        apply_bc ? c->cmask.p : nullptr, val);
    LAUNCH_CHECK(c, "k_jac2_blocks");
  }
  return MPM_OK;
}

// 3-D BSR blocks of context c from tangent records rec (indexed through pmap
// when given: record pmap[p] belongs to c's sorted particle p).
int launch_jac3_lines(mpm_ctx* c, const double* rec, const int32_t* pmap, double* val, bool apply_bc,
                      const int32_t* gstart) {
  const int64_t nwg = c->jl3_ws_h.empty() ? 0 : c->jl3_ws_h[c->nsim];
  if (nwg > 0 && c->n_row > 0) {
    k_jac3_lines<<<(unsigned)nwg, JL_T, 0, c->stream>>>(
        c->jl3_ws.p, c->nsim, c->sims.p, gstart ? gstart : c->gstart.p, c->node_map.p, rec, pmap, c->rowptr.p,
        c->slot.p, apply_bc ? c->bcode.p : nullptr, val);
    LAUNCH_CHECK(c, "k_jac3_lines");
  }
  return MPM_OK;
}

// 3-D tangent records at du into c->pdat3: the increment gradients and
// stencil weights once per particle, then the nine forward-mode lanes.
static int launch_tan3(mpm_ctx* c, const AsmArgs& A, const double* du) {
  if (c->pdat3.ensure(std::max<int64_t>(1, c->np) * PTW3) != hipSuccess ||
      c->pdF3.ensure(std::max<int64_t>(1, c->np) * 9) != hipSuccess)
    return c->fail(MPM_E_NOMEM, "3-D tangent records allocation failed");
  if (c->np == 0) return MPM_OK;
  k_dF3<<<nb256(c->np), 256, 0, c->stream>>>(A, du, c->pdF3.p, c->pdat3.p);
  LAUNCH_CHECK(c, "k_dF3");
  k_tan3v<<<(unsigned)((c->np + TP3 - 1) / TP3), TL3, 0, c->stream>>>(A, c->pdF3.p, c->pdat3.p, c->flag.p);
  LAUNCH_CHECK(c, "k_tan3v");
  return MPM_OK;
}

int launch_jacobian(mpm_ctx* c, const mpm_problem* pb, const double* du, double* val, bool apply_bc) {
  AsmArgs A = make_args(c, pb);
  const int nd = c->nd;
  if (c->dim == 2 && !c->up) {
    // tangent records, then one writer per block (no clearing needed)
    if (c->pdat.ensure(std::max<int64_t>(1, c->np) * PD2) != hipSuccess)
      return c->fail(MPM_E_NOMEM, "particle tangent records allocation failed");
    if (c->np > 0) {
      k_tan2<<<(unsigned)((4 * c->np + 255) / 256), 256, 0, c->stream>>>(A, du, c->pdat.p);
      LAUNCH_CHECK(c, "k_tan2");
    }
    c->tan_ready = true;
    GUARD(launch_jac2_records(c, val, apply_bc));
  } else if (c->dim == 2) {
    // u-p: 7x7 tangent records, then one writer per 3x3 block
    if (c->pdat.ensure(std::max<int64_t>(1, c->np) * PU2) != hipSuccess)
      return c->fail(MPM_E_NOMEM, "particle tangent records allocation failed");
    if (c->np > 0) {
      k_tan2up<<<(unsigned)((8 * c->np + 255) / 256), 256, 0, c->stream>>>(A, du, c->pdat.p);
      LAUNCH_CHECK(c, "k_tan2up");
    }
    GUARD(launch_jac2up_records(c, c->pdat.p, val, apply_bc));
  }
  if (c->dim == 3) {
    // tangent records, then the row segments of every x-line (each block written once)
    GUARD(launch_tan3(c, A, du));
    c->tan_ready = true;
    GUARD(launch_jac3_lines(c, c->pdat3.p, nullptr, val, apply_bc));
  }
  return MPM_OK;
}

// y = J x without the matrix (see k_jv3c).  records: compute the tangent
// records at du first (else reuse those of the last assembly at the same du).
int launch_jv(mpm_ctx* c, const mpm_problem* pb, const double* du, bool records, const double* x, double* y,
              bool apply_bc) {
  if (c->up) return c->fail(MPM_E_INVALID, "the matrix-free product covers single-phase problems");
  AsmArgs A = make_args(c, pb);
  const int nd = c->nd;
  const int64_t nv = c->n_row * nd;
  const uint8_t* cm = apply_bc ? c->cmask.p : nullptr;
  if (c->dim == 2) {
    if (records) {
      if (c->pdat.ensure(std::max<int64_t>(1, c->np) * PD2) != hipSuccess)
        return c->fail(MPM_E_NOMEM, "particle tangent records allocation failed");
      if (c->np > 0) {
        k_tan2<<<(unsigned)((4 * c->np + 255) / 256), 256, 0, c->stream>>>(A, du, c->pdat.p);
        LAUNCH_CHECK(c, "k_tan2");
      }
      c->tan_ready = true;
    } else if (!c->tan_ready) {
      return c->fail(MPM_E_INVALID, "no tangent records of this prepare to reuse");
    }
    if (c->rrec.ensure(std::max<int64_t>(1, c->np) * RD2) != hipSuccess)
      return c->fail(MPM_E_NOMEM, "residual records allocation failed");
    if (c->np > 0) {
      k_jv2_rec<<<nb256(c->np), 256, 0, c->stream>>>(c->np, c->sims.p, c->psim.p, c->node_map.p, c->pdat.p, cm,
                                                    c->xs.p, x, c->rrec.p);
      LAUNCH_CHECK(c, "k_jv2_rec");
    }
    if (c->n_row > 0) {
      k_fint2_rows<<<(unsigned)((c->n_row * RL2 + 255) / 256), 256, 0, c->stream>>>(c->n_row, nd, 0, c->rgrp.p,
                                                                                    c->rrec.p, y);
      LAUNCH_CHECK(c, "k_fint2_rows");
    }
  } else {
    if (records) {
      GUARD(launch_tan3(c, A, du));
      c->tan_ready = true;
    } else if (!c->tan_ready) {
      return c->fail(MPM_E_INVALID, "no tangent records of this prepare to reuse");
    }
    HIPC(c, hipMemsetAsync(y, 0, nv * sizeof(double), c->stream));
    const int nsim = c->nsim;
    for (int col = 0; col < 27 && c->np > 0; ++col) {
      const int64_t nwg = c->jf3_ws_h[(size_t)col * (nsim + 1) + nsim];
      if (nwg == 0) continue;
      k_jv3c<<<(unsigned)nwg, FT3, 0, c->stream>>>(col, c->jf3_ws.p + (size_t)col * (nsim + 1), nsim, c->sims.p,
                                                   c->gstart.p, c->node_map.p, c->xs.p, c->np, c->pdat3.p, cm, x, y);
      LAUNCH_CHECK(c, "k_jv3c");
    }
  }
  if (apply_bc && nv > 0) {
    k_jv_bc<<<nb256(nv), 256, 0, c->stream>>>(nv, c->cmask.p, x, y);
    LAUNCH_CHECK(c, "k_jv_bc");
  }
  return MPM_OK;
}

int launch_update(mpm_ctx* c, const mpm_problem* pb, const double* du, double* x, double* F, double* be) {
  AsmArgs A = make_args(c, pb);
  if (c->np == 0) return MPM_OK;
  if (c->dim == 2) k_update<2><<<nb256(c->np), 256, 0, c->stream>>>(A, du, c->perm.p, x, F, be, c->flag.p);
  else k_update<3><<<nb256(c->np), 256, 0, c->stream>>>(A, du, c->perm.p, x, F, be, c->flag.p);
  LAUNCH_CHECK(c, "k_update");
  return MPM_OK;
}
