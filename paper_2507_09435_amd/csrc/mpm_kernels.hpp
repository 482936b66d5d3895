// Shared declarations of the HIP kernels and the context of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mpm.h"
#include "mpm_device.hpp"

namespace mpm {

// Per-simulation grid constants (device copy).
struct SimDev {
  int32_t n[3];        // cells per axis
  int32_t nna[3];      // nodes per axis (n + 3)
  int32_t noa[3];      // stencil origins per axis (n + 1): o in [-1, n-1]
  int32_t dim;
  double h, inv_h;
  double x0[3];
  int64_t node_base;   // first full-grid node id of this sim
  int64_t okey_base;   // first origin key of this sim
  int64_t row_base;    // first compact row of this sim (after prepare)
  int64_t p_begin, p_end;
  int32_t shape;       // 0 quadratic B-spline, 1 cpGIMP
  double lp0[3];       // cpGIMP: initial half-width of the particle domain per axis
  const double* Fs;    // cpGIMP: sorted deformation gradients (the domain follows F_kk)
};

// Row blocks of the Krylov / elementwise kernels: a block never spans two sims.
struct RowBlock {
  int32_t sim;
  int32_t row0, row1;  // [row0, row1)
};

constexpr int ROWS_PER_BLOCK = 64;
constexpr int NQ = 4;               // reduction slots per row block

template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t m) {
    if (m <= n && p) return hipSuccess;
    if (p) { (void)hipFree(p); p = nullptr; n = 0; }
    size_t bytes = (m ? m : 1) * sizeof(T);
    hipError_t e = hipMalloc((void**)&p, bytes);
    if (e == hipSuccess) n = m;
    return e;
  }
  void release() { if (p) (void)hipFree(p); p = nullptr; n = 0; }
};

}  // namespace mpm

struct mpm_ctx;
namespace mpm {
// One coarse multigrid level: a child context on the coarsened grids, its
// Dirichlet mask, the map to the finest particle records, its vectors and
// the chunks (at most MG_CHUNK particles of one stencil group) of its
// group-block assembly.
// Device view of one level for the fused coarse tail of the V-cycle.
struct MgTailLevel {
  const int32_t* rowptr;
  const int32_t* colind;
  const double* val;        // level operator (BSR, 2x2 blocks)
  const double* dinv;       // inverted diagonal blocks
  const SimDev* sims;       // per sim: first row
  const uint8_t* cmask;     // constrained unknowns
  const int32_t* rtab;      // as the coarse side: per row the 9 finer rows it gathers (-1: none)
  const int32_t* ptab;      // as the fine side: per row the <= 4 coarser rows it takes (-1: none)
  const double* pw;         // as the fine side: per row the interpolation weight
  int32_t n_row;
  int32_t nsim;
  int32_t lds;              // LDS offset (doubles) of this level's vectors y, r, x, b
  int32_t ldn;              // doubles per LDS vector (2 x the most rows of one sim)
};

struct MgLevel {
  mpm_ctx* sub = nullptr;
  std::vector<mpm_grid> grids;
  DBuf<uint8_t> mask;        // full coarse grid [nodes][2]
  DBuf<int32_t> pmap;        // child-sorted particle -> finest-sorted particle
  DBuf<double> vec;          // sweep partner, residual, solution, right-hand side (4 * n_row * 2)
  DBuf<int32_t> chunk;       // per chunk: first particle, count
  DBuf<int32_t> key_chunk;   // per origin key: first chunk (n_okeys + 1)
  DBuf<double> part;         // per chunk: 81 partial 2x2 blocks
  int64_t n_chunks = 0;
  int32_t max_key_chunks = 0;   // most chunks of one origin key
  // 3x3-block levels: quadrature particles, NG per non-empty origin (at the
  // Gauss points of the origin's dual cell), carrying the origin's summed
  // tangent tables / NG
  DBuf<int32_t> pg;          // per origin key: first quadrature particle (n_okeys + 1)
  DBuf<int32_t> nek;         // non-empty origin keys
  DBuf<double> pxs;          // quadrature particle positions [dim][npp]
  DBuf<double> prec;         // quadrature particle records [npp][record]
  DBuf<int32_t> qsim;        // sim of each quadrature particle
  DBuf<int32_t> prgrp;       // plane strain: row group table over the quadrature particles
  int64_t npp = 0, n_nek = 0;
};
}  // namespace mpm

struct mpm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;

  // identity of the prepared problem
  bool prepared = false;
  int dim = 0, nd = 0, nsim = 0, up = 0, dp = 0;
  int64_t np = 0, n_nodes = 0, n_okeys = 0, n_row = 0, nnzb = 0;
  const double* user_x = nullptr;
  std::vector<mpm::SimDev> sims_h;
  std::vector<int64_t> sim_row_start;   // [nsim+1]
  std::vector<mpm::RowBlock> blocks_h;
  std::vector<int32_t> sim_blk_first;   // [nsim+1]

  // sorting / pattern
  mpm::DBuf<mpm::SimDev> sims;
  mpm::DBuf<int64_t> sim_start;
  mpm::DBuf<int32_t> okey, gcount, gstart, cursor, perm, psim;   // cursor: input indices between sort passes
  mpm::DBuf<int32_t> okey_sorted;
  mpm::DBuf<int32_t> sort_hist, sort_off;      // key sort: per (digit, tile) counts and their scan
  mpm::DBuf<int32_t> scan_tmp;
  mpm::DBuf<int32_t> node_flag, node_map;      // node_map: full node -> row or -1
  mpm::DBuf<int64_t> active_nodes;
  mpm::DBuf<int32_t> row_sim, rowcnt, rowptr, colind;
  mpm::DBuf<int8_t> slot;                      // [n_row][5^d] position in row or -1
  mpm::DBuf<int32_t> rgrp;                     // 2-D: [n_row][9][2] particle range of each stencil group
  mpm::DBuf<uint8_t> bcode;                    // 2-D, 2 unknowns: [n_row][25] constrained row (bits 2,3) / column (0,1) unknowns
  mpm::DBuf<mpm::RowBlock> blocks;
  mpm::DBuf<int32_t> blk_first;                // [nsim+1]
  mpm::DBuf<int32_t> flag;                     // device error flags

  // sorted particle copies
  mpm::DBuf<double> xs, vol0s, Fs, bes, Es, phis;

  // grid vectors (compact, n_row * nd)
  mpm::DBuf<uint8_t> cmask, rmask;
  mpm::DBuf<double> cval, fext, fint, nvol, work;
  mpm::DBuf<double> val, dinv;
  mpm::DBuf<double> pdat;                      // per-particle tangent records (2-D assembly)
  mpm::DBuf<double> pdat3;                     // per-particle tangent records (3-D assembly)
  mpm::DBuf<double> pdF3;                      // 3-D increment gradients dF per particle [9][np]
  bool tan_ready = false;                      // pdat / pdat3 hold this prepare's tangent records
  mpm::DBuf<int64_t> jc3_ws;                   // 3-D colour passes: per colour and sim, first workgroup
  std::vector<int64_t> jc3_ws_h;               // host staging of jc3_ws
  mpm::DBuf<int64_t> jf3_ws;                   // fused 3-D internal force: per colour and sim, first workgroup
  std::vector<int64_t> jf3_ws_h;               // host staging of jf3_ws
  mpm::DBuf<int64_t> jl3_ws;                   // 3-D line sweep: per sim, first workgroup
  std::vector<int64_t> jl3_ws_h;               // host staging of jl3_ws
  mpm::DBuf<double> gbuf;                      // per-origin group blocks (2-D assembly)
  mpm::DBuf<double> rrec;                      // per-particle residual records (2-D)
  // Krylov
  mpm::DBuf<double> kx, kr, krh, kp, kv, ks, kt, kph, ksh, kb;
  mpm::DBuf<double> part;                      // [nblocks][NQ]
  mpm::DBuf<double> simsc;                     // per-sim scalars [nsim][16]
  mpm::DBuf<int32_t> simflag;                  // per-sim krylov state [nsim][2]
  mpm::DBuf<double> gV, gsc, gpart;            // GMRES basis, per-sim Hessenberg/rotations, partials
  mpm::DBuf<int32_t> gflag;                    // per-sim GMRES state [nsim][2]
  mpm::DBuf<uint8_t> greset;
  int kmethod = 0;                             // 0: BiCGStab then GMRES fallback, 1: GMRES only
  bool kfused = true;                          // BiCGStab consumers sum the row-block partials themselves
  int spmv_lanes = 0;                          // lanes per BSR row picked by the autotuner (0: not yet)
  int spmv_pin = 0;                            // lanes per BSR row fixed by the caller (0: autotune)
  double kdec = 0.0;                           // residual decades per BiCGStab iteration, previous solve
  mpm::DBuf<double> du_base, alpha;            // line search
  // adjoint
  mpm::DBuf<int32_t> tpos;                     // position of the transposed block
  bool tpos_ready = false;
  bool ktrans = false;                         // Krylov on J^T
  mpm::DBuf<double> dinvT, adj_mu, adj_nu, adj_theta, adj_rbar;
  bool krylov_soft = false;                    // last solve stopped at its floor above rtol
  std::vector<double> kratio;                  // last solve: true relative residual per sim
  int time_spmv = 0;                           // sample period of SpMV timing (0: off)
  std::vector<hipEvent_t> spmv_events;
  double spmv_ms = 0.0;
  int64_t spmv_n = 0;
  double* host_pinned = nullptr;               // small pinned staging
  size_t host_pinned_n = 0;

  // multigrid hierarchy (levels 1..L are child contexts on grids of 2^l h)
  std::vector<mpm::MgLevel*> mgl;
  mpm::DBuf<double> mg_zero;                   // zero prescribed values for the child problems
  mpm::DBuf<int32_t> mg_inv;                   // finest sorted index of each original particle
  mpm::DBuf<double> mg_fine;                   // finest level: sweep partner and residual (2 * n_row * nd)
  mpm::DBuf<double> mg_dense;                  // coarsest level: per sim dense matrix and inverse
  mpm::DBuf<int32_t> mg_doff;                  // per sim: first coarsest row, rows
  mpm::DBuf<mpm::SimDev> mg_sims;              // staging of a child level's descriptors
  std::vector<double> mg3_lmax;                // 3x3-block levels: lambda_max(D^-1 A) per level and sim
  mpm::DBuf<double> mg3_lam;                   // (device copy)
  mpm::DBuf<double> mg3_inv;                   // power iteration: per sim 1 / ||w||
  mpm::DBuf<double> mg3_part;                  // power iteration: per row w.w
  mpm::DBuf<double> mg3_coef;                  // Chebyshev (c0, c1) per level, step and sim
  mpm::DBuf<int32_t> mg3_depth;                // 3x3-block levels: per sim, the level solved densely
  std::vector<int32_t> mg3_depth_h;            // (host copy; finer levels smooth the sim, coarser skip it)
  int mg_nmax = 0;                             // largest coarsest system (unknowns)
  bool mg_ready = false;                       // hierarchy built for the current prepare
  bool mg_on = false;                          // precondition the current solve with a V-cycle
  bool mg_level = false;                       // this context is a coarse multigrid level
  bool mg_graph = true;                        // replay captured V-cycles (false: launch them eagerly)
  uint64_t mg_gen = 0;                         // bumped whenever the hierarchy is rebuilt
  hipStream_t lstream = nullptr;               // stream the V-cycle kernels are launched on
  hipStream_t cap_stream = nullptr;            // private stream for graph capture
  struct MgGraph { hipGraphExec_t exec = nullptr; const void* key[5] = {}; uint64_t gen = 0; };
  MgGraph mg_exec[2];                          // V-cycles of BiCGStab's two preconditioner applications
  int mg_next = 0;
  int mg_tail_first = -1;                      // first level of the fused coarse tail (-1: none)
  bool mg_fuse = true;                         // run the coarse tail in one launch
  mpm::DBuf<mpm::MgTailLevel> mg_tail;         // tail levels' device views (first .. coarsest)
  std::vector<mpm::MgTailLevel> mg_tail_h;     // host staging of mg_tail
  mpm::DBuf<int32_t> mg_tab;                   // tail transfer tables (restriction 9, prolongation 4 per row)
  mpm::DBuf<double> mg_tabw;                   // tail prolongation weights
  std::vector<int64_t> mg_tab_off;             // per tail level: rtab, ptab, pw offsets (-1: none)
  std::vector<int64_t> mg_lvl_off;             // per level: rtab, ptab, pw offsets in mg_tab / mg_tabw (-1: none)
  int mg_tail_lds = 0;                         // bytes of LDS the tail kernel uses

  int fail(int code, const std::string& msg) { err = msg; return code; }
};
