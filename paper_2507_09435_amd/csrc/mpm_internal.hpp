// Internal helpers shared by the library's translation units.
#pragma once
#include <algorithm>
#include <cmath>
#include <string>

#include "mpm_kernels.hpp"

#define HIPC(c, x)                                                                              \
  do {                                                                                          \
    hipError_t e_ = (x);                                                                        \
    if (e_ != hipSuccess) return (c)->fail(MPM_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define GUARD(expr)          \
  do {                       \
    int rc_ = (expr);        \
    if (rc_) return rc_;     \
  } while (0)

#define LAUNCH_CHECK(c, name)                                                                   \
  do {                                                                                          \
    hipError_t e_ = hipGetLastError();                                                          \
    if (e_ != hipSuccess) return (c)->fail(MPM_E_HIP, std::string(name) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace mpm {

// B-spline stencil of one particle: per-axis origin, weights and gradients.
template <int DIM>
struct Stencil {
  static constexpr int NN = DIM == 2 ? 9 : 27;
  int32_t o[3];
  double w[3][3], dw[3][3];

  __device__ __forceinline__ int64_t node(const SimDev& S, int a) const {
    int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
    int64_t id = (o[0] + ax + 1) + (int64_t)S.nna[0] * (o[1] + ay + 1);
    if (DIM == 3) id += (int64_t)S.nna[0] * S.nna[1] * (o[2] + az + 1);
    return S.node_base + id;
  }
  __device__ __forceinline__ double weight(int a) const {
    double v = w[0][a % 3] * w[1][(a / 3) % 3];
    if (DIM == 3) v *= w[2][a / 9];
    return v;
  }
  __device__ __forceinline__ void grad(int a, double g[DIM]) const {
    int ax = a % 3, ay = (a / 3) % 3, az = a / 9;
    if (DIM == 2) {
      g[0] = dw[0][ax] * w[1][ay];
      g[1] = w[0][ax] * dw[1][ay];
    } else {
      g[0] = dw[0][ax] * w[1][ay] * w[2][az];
      g[1] = w[0][ax] * dw[1][ay] * w[2][az];
      g[2] = w[0][ax] * w[1][ay] * dw[2][az];
    }
  }
};

// Origin o = floor((x - x0)/h - 1/2) and xi = (x - x0)/h - o per axis.
template <int DIM>
__device__ __forceinline__ void make_stencil(const SimDev& S, const double* __restrict__ xs, int64_t np, int64_t i,
                                             Stencil<DIM>& st) {
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    double u = (xs[k * np + i] - S.x0[k]) / S.h;
    double of = floor(u - 0.5);
    st.o[k] = (int32_t)of;
    if (S.shape == 1) {
      // the particle domain follows the stretch of its axis: l = lp0 F_kk
      const double l = S.lp0[k] * S.Fs[(k * DIM + k) * np + i] * S.inv_h;
      gimp3(u - of, l, S.inv_h, st.w[k], st.dw[k]);
    } else {
      bspline3<double>(u - of, S.inv_h, st.w[k], st.dw[k]);
    }
  }
  if (DIM == 2) {
    st.o[2] = 0;
    st.w[2][0] = st.w[2][1] = st.w[2][2] = 1.0;
    st.dw[2][0] = st.dw[2][1] = st.dw[2][2] = 0.0;
  }
}

// Offset index of node b relative to node a inside the 5^d neighbourhood.
template <int DIM>
__device__ __forceinline__ int nb_index(int a, int b) {
  int dx = b % 3 - a % 3 + 2, dy = (b / 3) % 3 - (a / 3) % 3 + 2;
  if (DIM == 2) return dx + 5 * dy;
  int dz = b / 9 - a / 9 + 2;
  return dx + 5 * dy + 25 * dz;
}

}  // namespace mpm

namespace mpm {
constexpr int PD2 = 32;       // doubles per 2-D particle record: V0 T 0..15, wx 16..18, dwx 19..21, wy 22..24, dwy 25..27
constexpr int PT3 = 81;       // 3-D tangent table: V0 dP_ri/dF_cj at (r * 3 + c) * 9 + i * 3 + j
constexpr int PTW3 = 99;      // doubles per 3-D tangent record: the table, then per axis k the weights
                              // at PT3 + 6 k + 0..2 and their derivatives at PT3 + 6 k + 3..5
constexpr int PU2 = 64;       // doubles per u-p record: V0 T 0..48 (7x7), wx 49..51, dwx 52..54, wy 55..57, dwy 58..60
constexpr int GB2 = 81 * 4;   // doubles per origin in the 2-D group-block buffer
}  // namespace mpm

int validate_problem(mpm_ctx* c, const mpm_problem* pb);
int check_prepared(mpm_ctx* c, const mpm_problem* pb);
int mpm_prepare_impl(mpm_ctx* c, const mpm_problem* pb, int64_t* n_row, int64_t* nnzb, int32_t* nd);
namespace mpm {
int scan_excl(mpm_ctx* c, const int32_t* in, int64_t n, int32_t* out, int32_t* total);
}
int sim_sum_launch(mpm_ctx* c, const double* part, int q, int off);
int64_t fint_record_doubles(int dim);
int launch_fint(mpm_ctx* c, const mpm_problem* pb, const double* du, double* rec = nullptr);
int launch_residual(mpm_ctx* c, const mpm_problem* pb, const double* du, double* r, double* r_raw,
                    double* rec = nullptr);
int launch_jacobian(mpm_ctx* c, const mpm_problem* pb, const double* du, double* val, bool apply_bc);
// gstart: particle ranges per origin to use in place of c's own (the
// quadrature particles of a multigrid level, whose records are in level order)
int launch_jac3_lines(mpm_ctx* c, const double* rec, const int32_t* pmap, double* val, bool apply_bc,
                      const int32_t* gstart = nullptr);
int launch_row_groups(mpm_ctx* c, const int32_t* gstart, int32_t* rgrp);
int launch_jv(mpm_ctx* c, const mpm_problem* pb, const double* du, bool records, const double* x, double* y,
              bool apply_bc);
int launch_update(mpm_ctx* c, const mpm_problem* pb, const double* du, double* x, double* F, double* be);
int launch_bj_inv(mpm_ctx* c, const double* val);
int launch_spmv(mpm_ctx* c, const double* val, const double* x, double* y, const double* z);
int krylov_solve(mpm_ctx* c, const double* val, double rtol, int max_iter, std::vector<int>& iters_out);
int launch_jac2_records(mpm_ctx* c, double* val, bool apply_bc);
int launch_jac2up_records(mpm_ctx* c, const double* rec, double* val, bool apply_bc, const int32_t* rgrp = nullptr);
int build_colour_table(mpm_ctx* c);
int launch_p2g3(mpm_ctx* c, int mode, const double* rec, double* out);
int launch_jac2_blocks(mpm_ctx* c, double* val, bool apply_bc);
void ctx_release(mpm_ctx* c);
// multigrid preconditioner (single-phase; the 3-D levels in mpm_mg3.hip)
int mg_build(mpm_ctx* c, const mpm_problem* pb);
int mg_setup(mpm_ctx* c);
int mg_vcycle(mpm_ctx* c, const double* b, double* x);
void mg_release(mpm_ctx* c);
void mg_drop_graphs(mpm_ctx* c);
void mg_level_release(mpm::MgLevel* L);
int mg3_build(mpm_ctx* c, const mpm_problem* pb);
int mg3_setup(mpm_ctx* c);
int mg3_vcycle(mpm_ctx* c, const double* b, double* x);
