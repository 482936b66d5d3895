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
  int nd, up, dp, match;
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
    for (int a = 0; a < Stencil<DIM>::NN; ++a) {
      int32_t r = A.node_map[L.st.node(S, a)];
      L.row[a] = r;
      double g[DIM];
      L.st.grad(a, g);
      const double* u = du + (int64_t)r * nd;
#pragma unroll
      for (int q = 0; q < DIM; ++q) {
        double uq = u[q];
#pragma unroll
        for (int k = 0; k < DIM; ++k) L.dF[q][k] += uq * g[k];
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
  Mat<dnum> m = make_mat<dnum>(dnum(L.E), A.nu, dnum(L.phi), A.c, A.psi, A.dp, A.match, A.apex_reg);
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
  mech2<dnum>(m, F, bd, dnum(L.Jn), NIO == 7, u, pp, gp, o, nullptr);
  Tc[0] = o.P[0][0].d; Tc[1] = o.P[0][1].d; Tc[2] = o.P[1][0].d; Tc[3] = o.P[1][1].d;
  if constexpr (NIO == 7) { Tc[4] = o.s1.d; Tc[5] = o.vv[0].d; Tc[6] = o.vv[1].d; }
}

// ---------------------------------------------- group-cooperative 2-D ------
// Particles of one stencil group (same origin) are adjacent after sorting.
// A workgroup stages per-particle data in LDS, finds the group starts with a
// ballot scan, and then one thread per (group, node) sums the group's
// contributions in registers before a single atomic per entry.
constexpr int GP = 128;   // particles (threads) per workgroup

__device__ __forceinline__ int32_t origin_key2(const SimDev& S, const Stencil<2>& st) {
  return (int32_t)(S.okey_base + (st.o[0] + 1) + (int64_t)S.noa[0] * (st.o[1] + 1));
}

// Group starts of the workgroup's particles (n valid).  Returns the number of
// groups; gstart[g] = first local index of group g, gstart[G] = n.
__device__ __forceinline__ int group_starts(const int32_t* key, int n, int32_t* gstart, int32_t* wave_cnt) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  bool head = t < n && (t == 0 || key[t] != key[t - 1]);
  unsigned long long m = __ballot(head);
  int before = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) wave_cnt[wv] = __popcll(m);
  __syncthreads();
  int off = 0;
  for (int w = 0; w < wv; ++w) off += wave_cnt[w];
  if (head) gstart[off + before] = t;
  int G = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) G += wave_cnt[w];
  if (t == 0) gstart[G] = n;
  __syncthreads();
  return G;
}

// 2-D Jacobian.  Phase 1: LP lanes per particle, lane q computes tangent
// column q (one forward pass each), so a workgroup holds JP particles and a
// small problem still fills the chip.  Phase 2: one thread per (group,
// column node b, row of 3 nodes a) sums the group's contributions to its
// three local blocks in registers, then adds each entry once.
constexpr int JT = 256;                       // threads per workgroup

template <int NIO>
__global__ void __launch_bounds__(JT) k_jac2g(AsmArgs A, const double* __restrict__ du,
                                             const int32_t* __restrict__ rowptr, const int8_t* __restrict__ slot,
                                             double* __restrict__ val) {
  constexpr int ND = NIO == 7 ? 3 : 2;
  constexpr int LP = NIO == 7 ? 8 : 4;       // lanes per particle in phase 1
  constexpr int JP = JT / LP;                 // particles per workgroup
  __shared__ double sT[JP][NIO * NIO];        // V0 * tangent table
  __shared__ double sW[JP][2][3], sD[JP][2][3];
  __shared__ int32_t sKey[JP], sRow[JP][9], sG[JP + 1], sWc[JT / 64];
  const int64_t base = (int64_t)blockIdx.x * JP;
  const int n = (int)min<int64_t>(JP, A.np - base);
  const int t = threadIdx.x;
  const int lp = t / LP, q = t % LP;
  if (lp < n && q < NIO) {
    const int64_t i = base + lp;
    PLoad<2> L;
    load_particle<2>(A, i, du, L);
    double Tc[NIO];
    tangent2_col<NIO>(A, L, load_be2(A, i), q, Tc);
#pragma unroll
    for (int o = 0; o < NIO; ++o) sT[lp][o * NIO + q] = L.v0 * Tc[o];
    if (q == 0) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) { sW[lp][k][a] = L.st.w[k][a]; sD[lp][k][a] = L.st.dw[k][a]; }
#pragma unroll
      for (int a = 0; a < 9; ++a) sRow[lp][a] = L.row[a];
      sKey[lp] = origin_key2(A.sims[A.psim[i]], L.st);
    }
  }
  __syncthreads();
  const int G = group_starts(sKey, n, sG, sWc);
  for (int task = t; task < 27 * G; task += JT) {
    const int g = task / 27, rem = task % 27, b = rem % 9, ay = rem / 9;
    const int bx = b % 3, by = b / 3;
    double acc[3][ND][ND];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int r = 0; r < ND; ++r)
#pragma unroll
        for (int c = 0; c < ND; ++c) acc[a][r][c] = 0.0;
    for (int p = sG[g]; p < sG[g + 1]; ++p) {
      const double* T = sT[p];
      const double gb0 = sD[p][0][bx] * sW[p][1][by], gb1 = sW[p][0][bx] * sD[p][1][by];
      double Tb[NIO][ND];
#pragma unroll
      for (int o = 0; o < NIO; ++o) {
#pragma unroll
        for (int m = 0; m < 2; ++m) Tb[o][m] = T[o * NIO + m * 2] * gb0 + T[o * NIO + m * 2 + 1] * gb1;
        if constexpr (ND == 3) {
          const double wb = sW[p][0][bx] * sW[p][1][by];
          Tb[o][2] = T[o * NIO + 4] * wb + T[o * NIO + 5] * gb0 + T[o * NIO + 6] * gb1;
        }
      }
      const double wy = sW[p][1][ay], dy = sD[p][1][ay];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const double ga0 = sD[p][0][ax] * wy, ga1 = sW[p][0][ax] * dy;
#pragma unroll
        for (int c = 0; c < ND; ++c) {
#pragma unroll
          for (int r = 0; r < 2; ++r) acc[ax][r][c] += ga0 * Tb[r * 2][c] + ga1 * Tb[r * 2 + 1][c];
          if constexpr (ND == 3) {
            const double wa = sW[p][0][ax] * wy;
            acc[ax][2][c] += wa * Tb[4][c] + ga0 * Tb[5][c] + ga1 * Tb[6][c];
          }
        }
      }
    }
    const int p0 = sG[g];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int a = ay * 3 + ax;
      const int32_t ra = sRow[p0][a];
      const int s = slot[(int64_t)ra * 25 + nb_index<2>(a, b)];
      double* blk = val + ((int64_t)rowptr[ra] + s) * (ND * ND);
#pragma unroll
      for (int r = 0; r < ND; ++r)
#pragma unroll
        for (int c = 0; c < ND; ++c) atomicAdd(&blk[r * ND + c], acc[ax][r][c]);
    }
  }
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

// 3-D Jacobian without atomics.  k_tan3: one thread per particle writes its
// tangent table (V0 dP/dF, 81 entries, from 9 forward passes) and its
// stencil weights and derivatives to a record.  k_jac3c: stencil groups of
// one colour (origin index mod 3 per axis) hold pairwise disjoint node sets,
// so one workgroup per group adds its 729 3x3 blocks with plain
// read-modify-writes; the 27 colours run in a fixed order, every group's
// particles in order, so the result is deterministic.
constexpr int PD3 = 100;   // doubles per 3-D record: T 0..80 ((r*3+c)*9 + q), w 81..89 [axis][a], dw 90..98
constexpr int JC3 = 32;    // records staged in LDS at a time

__global__ void __launch_bounds__(GP3) k_tan3(AsmArgs A, const double* __restrict__ du, double* __restrict__ rec,
                                              int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * GP3 + threadIdx.x;
  if (i >= A.np) return;
  PLoad<3> L;
  load_particle<3>(A, i, du, L);
  Mat<dnum> m = make_mat<dnum>(dnum(L.E), A.nu, dnum(L.phi), A.c, A.psi, A.dp, A.match, A.apex_reg);
  Sym3<double> be = load_be3(A, i);
  double* R = rec + i * PD3;
  int rerr = 0;
  for (int q = 0; q < 9; ++q) {
    dnum F[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) F[r][c] = dnum(L.dF[r][c], q == r * 3 + c ? 1.0 : 0.0);
    Sym3<dnum> bd;
#pragma unroll
    for (int k = 0; k < 6; ++k) bd.a[k] = dnum(be.a[k]);
    Out3<dnum> o;
    mech3<dnum>(m, F, bd, o, nullptr, &rerr);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) R[(r * 3 + c) * 9 + q] = L.v0 * o.P[r][c].d;
  }
  if (rerr) atomicOr(flag, 4);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      R[81 + k * 3 + a] = L.st.w[k][a];
      R[90 + k * 3 + a] = L.st.dw[k][a];
    }
}

// Origins of colour (cx, cy, cz) along one axis: v = o + 1 in [0, n] with v = c mod 3.
__device__ __host__ __forceinline__ int colour_count(int n, int c) { return c > n ? 0 : (n - c) / 3 + 1; }

constexpr int JC3T = 256;   // threads: task t < 243 is (column node b, z-layer of a, block row r)
__global__ void __launch_bounds__(JC3T) k_jac3c(int colour, const int64_t* __restrict__ wstart, int nsim,
                                                const SimDev* __restrict__ sims, const int32_t* __restrict__ gstart,
                                                const int32_t* __restrict__ node_map, const double* __restrict__ rec,
                                                const int32_t* __restrict__ rowptr, const int8_t* __restrict__ slot,
                                                double* __restrict__ val) {
  __shared__ double sT[JC3][81];
  __shared__ double sW[JC3][3][3], sD[JC3][3][3];
  __shared__ int32_t sRow[27];
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
  if (t < 27) {
    const int ax = t % 3, ay = (t / 3) % 3, az = t / 9;
    sRow[t] = node_map[S.node_base + (ox + ax + 1) + (int64_t)S.nna[0] * ((oy + ay + 1) + (int64_t)S.nna[1] * (oz + az + 1))];
  }
  const bool task = t < 243;
  const int r = t % 3, az = (t / 3) % 3, b = t / 9;
  const int bx = b % 3, by = (b / 3) % 3, bz = b / 9;
  double acc[9][3];
#pragma unroll
  for (int a = 0; a < 9; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[a][c] = 0.0;
  for (int c0 = p0; c0 < p1; c0 += JC3) {
    const int nc = min(JC3, p1 - c0);
    __syncthreads();   // the previous chunk is consumed
    for (int e = t; e < nc * 99; e += JC3T) {
      const int q = e / 99, k = e % 99;
      const double v = rec[(int64_t)(c0 + q) * PD3 + k];
      if (k < 81) sT[q][k] = v;
      else if (k < 90) sW[q][(k - 81) / 3][(k - 81) % 3] = v;
      else sD[q][(k - 90) / 3][(k - 90) % 3] = v;
    }
    __syncthreads();
    if (task) {
      for (int p = 0; p < nc; ++p) {
        const double* T = sT[p];
        const double gb0 = sD[p][0][bx] * sW[p][1][by] * sW[p][2][bz];
        const double gb1 = sW[p][0][bx] * sD[p][1][by] * sW[p][2][bz];
        const double gb2 = sW[p][0][bx] * sW[p][1][by] * sD[p][2][bz];
        double Tb[3][3];   // Tb[i][c] = sum_j dP_{r i}/dF_{c j} grad_j w_b
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const double* Tq = T + (r * 3 + i) * 9 + c * 3;
            Tb[i][c] = Tq[0] * gb0 + Tq[1] * gb1 + Tq[2] * gb2;
          }
#pragma unroll
        for (int a = 0; a < 9; ++a) {
          const int ax = a % 3, ay = a / 3;
          const double ga0 = sD[p][0][ax] * sW[p][1][ay] * sW[p][2][az];
          const double ga1 = sW[p][0][ax] * sD[p][1][ay] * sW[p][2][az];
          const double ga2 = sW[p][0][ax] * sW[p][1][ay] * sD[p][2][az];
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[a][c] += ga0 * Tb[0][c] + ga1 * Tb[1][c] + ga2 * Tb[2][c];
        }
      }
    }
  }
  if (task) {
#pragma unroll
    for (int a9 = 0; a9 < 9; ++a9) {
      const int a = a9 + 9 * az;
      const int32_t ra = sRow[a];
      const int sl = slot[(int64_t)ra * 125 + nb_index<3>(a, b)];
      double* blk = val + ((int64_t)rowptr[ra] + sl) * 9 + r * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) blk[c] += acc[a9][c];   // one writer per entry in this colour
    }
  }
}

// 3-D internal force without atomics: k_fint3_rec writes per particle V0 P
// and the stencil weights and derivatives; k_p2g3c (shared with the
// external force) gives one workgroup to each stencil group of a colour and
// adds the group's sum over its particles, in order, to each of its 27
// nodes with a plain read-modify-write.
constexpr int PR3 = 28;    // doubles per 3-D force record: V0 P 0..8 (or the force 0..2), w 9..17 [axis][a], dw 18..26

__global__ void __launch_bounds__(256) k_fint3_rec(AsmArgs A, const double* __restrict__ du, double* __restrict__ rec,
                                                  int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= A.np) return;
  PLoad<3> L;
  load_particle<3>(A, i, du, L);
  Mat<double> m = make_mat<double>(L.E, A.nu, L.phi, A.c, A.psi, A.dp, A.match, A.apex_reg);
  Out3<double> o;
  int rerr = 0;
  mech3<double>(m, L.dF, load_be3(A, i), o, nullptr, &rerr);
  if (rerr) atomicOr(flag, 4);
  double* R = rec + i * PR3;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) R[r * 3 + c] = L.v0 * o.P[r][c];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      R[9 + k * 3 + a] = L.st.w[k][a];
      R[18 + k * 3 + a] = L.st.dw[k][a];
    }
}

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

// Dirichlet rows/columns: zero them, 1 on the diagonal (structure unchanged).
__global__ void k_jac_bc(int64_t n_row, int nd, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                         const uint8_t* __restrict__ cmask, double* __restrict__ val) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_row) return;
  for (int32_t k = rowptr[r]; k < rowptr[r + 1]; ++k) {
    int32_t c = colind[k];
    double* blk = val + (int64_t)k * nd * nd;
    for (int i = 0; i < nd; ++i)
      for (int j = 0; j < nd; ++j)
        if (cmask[r * nd + i] || cmask[(int64_t)c * nd + j]) blk[i * nd + j] = (r == c && i == j) ? 1.0 : 0.0;
  }
}

// ------------------------------------------------------------- update ------
template <int DIM>
__global__ void k_update(AsmArgs A, const double* __restrict__ du, const int32_t* __restrict__ perm,
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
    Sym2<double> ee;
    double F[2][2] = {{L.dF[0][0], L.dF[0][1]}, {L.dF[1][0], L.dF[1][1]}};
    double gp0[2] = {0.0, 0.0};
    mech2<double>(m, F, load_be2(A, i), L.Jn, 0, up_par(A), 0.0, gp0, o, &ee);
    Sym2<double> b = exp2eps2(ee);
    if (be_out) {
      be_out[0 * np + p] = b.xx; be_out[1 * np + p] = b.yy; be_out[2 * np + p] = b.xy; be_out[3 * np + p] = b.zz;
    }
  } else {
    Out3<double> o;
    Sym3<double> ee;
    int rerr = 0;
    mech3<double>(m, L.dF, load_be3(A, i), o, &ee, &rerr);
    if (rerr) atomicOr(flag, 4);
    Sym3<double> b = exp2eps3(ee);
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
int64_t fint_record_doubles(int dim) { return dim == 2 ? RD2 : PR3; }

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
  // force records, then the 27 colours of stencil groups in order
  k_fint3_rec<<<(unsigned)((c->np + 255) / 256), 256, 0, c->stream>>>(A, du, rec, c->flag.p);
  LAUNCH_CHECK(c, "k_fint3_rec");
  return launch_p2g3(c, 0, rec, c->fint.p);
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
    GUARD(launch_jac2_records(c, val, apply_bc));
  } else {
    HIPC(c, hipMemsetAsync(val, 0, c->nnzb * nd * nd * sizeof(double), c->stream));
  }
  if (c->np > 0 && c->dim == 2 && c->up) {
    const unsigned g8 = (unsigned)((c->np + JT / 8 - 1) / (JT / 8));
    k_jac2g<7><<<g8, JT, 0, c->stream>>>(A, du, c->rowptr.p, c->slot.p, val);
    LAUNCH_CHECK(c, "k_jac2g");
  }
  if (c->np > 0 && c->dim == 3) {
    // tangent records, then the 27 colours of stencil groups in order
    if (c->pdat3.ensure(c->np * PD3) != hipSuccess)
      return c->fail(MPM_E_NOMEM, "3-D tangent records allocation failed");
    k_tan3<<<(unsigned)((c->np + GP3 - 1) / GP3), GP3, 0, c->stream>>>(A, du, c->pdat3.p, c->flag.p);
    LAUNCH_CHECK(c, "k_tan3");
    const int nsim = c->nsim;
    for (int col = 0; col < 27; ++col) {
      const int64_t nwg = c->jc3_ws_h[(size_t)col * (nsim + 1) + nsim];
      if (nwg == 0) continue;
      k_jac3c<<<(unsigned)nwg, JC3T, 0, c->stream>>>(col, c->jc3_ws.p + (size_t)col * (nsim + 1), nsim, c->sims.p,
                                                      c->gstart.p, c->node_map.p, c->pdat3.p, c->rowptr.p, c->slot.p,
                                                      val);
      LAUNCH_CHECK(c, "k_jac3c");
    }
  }
  if (apply_bc && c->n_row > 0 && !(c->dim == 2 && !c->up)) {   // the 2-D single-phase writer applies it itself
    k_jac_bc<<<nb256(c->n_row), 256, 0, c->stream>>>(c->n_row, nd, c->rowptr.p, c->colind.p, c->cmask.p, val);
    LAUNCH_CHECK(c, "k_jac_bc");
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
