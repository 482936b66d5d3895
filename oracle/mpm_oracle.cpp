// Plain FP64 CPU oracle for the implicit-MPM Newton-iteration hot path.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
// calls this file; only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark do. It shares no code with the GPU path.
//
// What it computes, in the paper's order (arXiv 2507.09435, "GeoWarp"):
//   * particle-to-grid / grid-to-particle transfers with tensor-product
//     weights (Sec. 2.2, the four-stage update and the mass-weighted mapping
//     equation); the weights are quadratic B-splines (Sec. 3.2, Table 1:
//     support w = 3, Jacobian block width b = 2w - 1 = 5);
//   * finite-deformation kinematics F = 1 + du/dX, J = det F (Sec. 2.1);
//   * internal / external force vectors and the residual
//     r = A_p (f_int,p - f_ext,p) (Sec. 2.2, the discrete weak form and the
//     backward-Euler residual equation);
//   * the Jacobian J = dr/du (Sec. 2.2).  The paper obtains it by
//     reverse-mode AD with coloured seeds (Sec. 3.2, Alg. 2).  Here the same
//     matrix is obtained plainly: forward-mode dual numbers seeded on the
//     3^d * ndof local unknowns of one particle (local blocks, then a plain
//     scatter) and, for tiny grids, on every global unknown one at a time
//     (the dense analogue of Alg. 1).
//   * Hencky elasticity (Sec. 4.2 names it; the formula is the textbook one:
//     tau = lambda tr(eps) 1 + 2 mu eps, eps = 1/2 ln b^e) and a
//     Drucker-Prager return map in Kirchhoff-stress / log-strain space (not in
//     the paper; textbook plasticity cited in Sec. 2.1).
//   * u-p poromechanics terms (Sec. 2.2, Remark 1; the paper defers the
//     equations to its reference, the reading used here is a backward-Euler
//     fluid mass balance with Darcy flow and incompressible constituents).
//
// Everything is written generically over a scalar type T: T = double gives
// values, T = Dual<N> gives N directional derivatives in one pass.
//
// Parity notes: the matrix logarithm is evaluated without eigenvectors
// (inverse scaling and squaring with Denman-Beavers square roots and the
// Gregory series ln B = 2 atanh((B-1)(B+1)^-1)), so dual numbers stay finite
// at repeated eigenvalues (b^e = 1 in the undeformed state).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <vector>

namespace orc {

// ---------------------------------------------------------------- scalars --
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) { for (int k = 0; k < N; ++k) d[k] = 0.0; }
  Dual(double x) : v(x) { for (int k = 0; k < N; ++k) d[k] = 0.0; }
};

inline double val(double x) { return x; }
template <int N> inline double val(const Dual<N>& x) { return x.v; }

template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v; for (int k = 0; k < N; ++k) r.d[k] = -a.d[k]; return r; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
  return r; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> inline Dual<N> operator+(double b, const Dual<N>& a) { Dual<N> r = a; r.v += b; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> inline Dual<N> operator-(double b, const Dual<N>& a) { return Dual<N>(b) - a; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r; r.v = a.v * b; for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b; return r; }
template <int N> inline Dual<N> operator*(double b, const Dual<N>& a) { return a * b; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> inline Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N> inline Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) { a = a - b; return a; }

// chain rule helper: f(a) with value fv and derivative dfv
template <int N> inline Dual<N> chain(const Dual<N>& a, double fv, double dfv) {
  Dual<N> r; r.v = fv; for (int k = 0; k < N; ++k) r.d[k] = dfv * a.d[k]; return r; }
template <int N> inline Dual<N> sqrt(const Dual<N>& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int N> inline Dual<N> log(const Dual<N>& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
template <int N> inline Dual<N> exp(const Dual<N>& a) { double e = std::exp(a.v); return chain(a, e, e); }
template <int N> inline Dual<N> sin(const Dual<N>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <int N> inline Dual<N> cos(const Dual<N>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <int N> inline Dual<N> tan(const Dual<N>& a) { double c = std::cos(a.v); return chain(a, std::tan(a.v), 1.0 / (c * c)); }
using std::sqrt; using std::log; using std::exp; using std::sin; using std::cos; using std::tan;

// value of a, derivatives of b scaled by f (identity on plain doubles)
inline double with_derivative(double a, double, double) { return a; }
template <int N> inline Dual<N> with_derivative(const Dual<N>& a, const Dual<N>& b, double f) {
  Dual<N> r; r.v = a.v; for (int k = 0; k < N; ++k) r.d[k] = f * b.d[k]; return r; }

// ---------------------------------------------------------------- 3x3 -------
template <class T>
struct M3 {
  T a[3][3];
  static M3 zero() { M3 m; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) m.a[i][j] = T(0.0); return m; }
  static M3 eye() { M3 m = zero(); for (int i = 0; i < 3; ++i) m.a[i][i] = T(1.0); return m; }
};
template <class T> M3<T> mul(const M3<T>& A, const M3<T>& B) {
  M3<T> C = M3<T>::zero();
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) for (int k = 0; k < 3; ++k) C.a[i][j] += A.a[i][k] * B.a[k][j];
  return C; }
template <class T> M3<T> transpose(const M3<T>& A) {
  M3<T> C; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) C.a[i][j] = A.a[j][i]; return C; }
template <class T> M3<T> add(const M3<T>& A, const M3<T>& B) {
  M3<T> C; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) C.a[i][j] = A.a[i][j] + B.a[i][j]; return C; }
template <class T> M3<T> sub(const M3<T>& A, const M3<T>& B) {
  M3<T> C; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) C.a[i][j] = A.a[i][j] - B.a[i][j]; return C; }
template <class T, class S> M3<T> scale(const M3<T>& A, const S& s) {
  M3<T> C; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) C.a[i][j] = A.a[i][j] * s; return C; }
template <class T> T trace(const M3<T>& A) { return A.a[0][0] + A.a[1][1] + A.a[2][2]; }
template <class T> T det(const M3<T>& A) {
  return A.a[0][0] * (A.a[1][1] * A.a[2][2] - A.a[1][2] * A.a[2][1])
       - A.a[0][1] * (A.a[1][0] * A.a[2][2] - A.a[1][2] * A.a[2][0])
       + A.a[0][2] * (A.a[1][0] * A.a[2][1] - A.a[1][1] * A.a[2][0]); }
template <class T> M3<T> inverse(const M3<T>& A) {
  // adjugate / determinant
  M3<T> C;
  C.a[0][0] = A.a[1][1] * A.a[2][2] - A.a[1][2] * A.a[2][1];
  C.a[0][1] = A.a[0][2] * A.a[2][1] - A.a[0][1] * A.a[2][2];
  C.a[0][2] = A.a[0][1] * A.a[1][2] - A.a[0][2] * A.a[1][1];
  C.a[1][0] = A.a[1][2] * A.a[2][0] - A.a[1][0] * A.a[2][2];
  C.a[1][1] = A.a[0][0] * A.a[2][2] - A.a[0][2] * A.a[2][0];
  C.a[1][2] = A.a[0][2] * A.a[1][0] - A.a[0][0] * A.a[1][2];
  C.a[2][0] = A.a[1][0] * A.a[2][1] - A.a[1][1] * A.a[2][0];
  C.a[2][1] = A.a[0][1] * A.a[2][0] - A.a[0][0] * A.a[2][1];
  C.a[2][2] = A.a[0][0] * A.a[1][1] - A.a[0][1] * A.a[1][0];
  T d = det(A);
  return scale(C, T(1.0) / d); }
template <class T> double fro_val(const M3<T>& A) {
  double s = 0; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) s += val(A.a[i][j]) * val(A.a[i][j]); return std::sqrt(s); }

// ------------------------------------------------- matrix log / exp (SPD) ---
// ln A for symmetric positive-definite A, eigenvector-free:
//   A = c * B with c = det(A)^(1/3)            -> ln A = ln(c) 1 + ln B
//   B <- B^(1/2) (Denman-Beavers) s times until ||B - 1|| is small
//   ln B = 2^s * 2 * sum_{k odd} Z^k / k,  Z = (B - 1)(B + 1)^-1
template <class T> M3<T> sqrtm_db(const M3<T>& A) {
  M3<T> Y = A, Z = M3<T>::eye();
  int extra = -1;
  for (int it = 0; it < 100; ++it) {
    M3<T> Yn = scale(add(Y, inverse(Z)), 0.5);
    M3<T> Zn = scale(add(Z, inverse(Y)), 0.5);
    double change = fro_val(sub(Yn, Y)), size = fro_val(Yn);
    Y = Yn; Z = Zn;
    if (extra < 0 && change <= 1e-15 * size) extra = 2;  // two more sweeps so tangents settle too
    if (extra >= 0 && extra-- == 0) break;
  }
  return Y; }

template <class T> M3<T> logm_spd(const M3<T>& A) {
  T dA = det(A);
  T lnc = log(dA) / 3.0;
  M3<T> B = scale(A, exp(-lnc));
  int s = 0;
  const M3<T> I = M3<T>::eye();
  while (fro_val(sub(B, I)) > 0.25 && s < 60) { B = sqrtm_db(B); ++s; }
  M3<T> Z = mul(sub(B, I), inverse(add(B, I)));
  M3<T> Z2 = mul(Z, Z);
  M3<T> term = Z, sum = Z;
  double z1 = fro_val(Z);
  for (int k = 3; k < 400; k += 2) {
    term = mul(term, Z2);
    M3<T> t = scale(term, 1.0 / k);
    sum = add(sum, t);
    if (fro_val(t) <= 1e-19 * (z1 + 1e-300)) break;
  }
  double f = 2.0 * std::ldexp(1.0, s);
  M3<T> L = scale(sum, f);
  for (int i = 0; i < 3; ++i) L.a[i][i] += lnc;
  return L; }

// exp A for symmetric A: scaling and squaring around a Taylor series
template <class T> M3<T> expm_sym(const M3<T>& A) {
  int s = 0;
  double n = fro_val(A);
  while (n > 0.125 && s < 60) { n *= 0.5; ++s; }
  M3<T> As = scale(A, std::ldexp(1.0, -s));
  M3<T> term = M3<T>::eye(), sum = M3<T>::eye();
  for (int k = 1; k < 60; ++k) {
    term = scale(mul(term, As), 1.0 / k);
    sum = add(sum, term);
    if (fro_val(term) <= 1e-20) break;
  }
  for (int i = 0; i < s; ++i) sum = mul(sum, sum);
  return sum; }

// ------------------------------------------------------------- problem ----
struct Cfg {
  int32_t dim;       // 2 (plane strain) or 3
  int32_t up;        // 1: u-p poromechanics (extra nodal pressure unknown)
  int32_t dp;        // 1: Drucker-Prager plasticity on top of Hencky
  int32_t dp_match;  // 0 outer cone, 1 plane-strain match, 2 inner cone (bit 4: associated flow)
  int32_t n[3];      // cells per axis; nodes are -1 .. n+1 per axis
  double h;          // cell size
  double x0[3];      // grid origin (coordinate of node 0)
  double E, nu, phi, c, psi;  // defaults when no per-particle array is given
  double rho0, g[3];
  double perm, mu_f, biot, rho_f, dt;
  double apex_reg;   // tangent of an apex return = apex_reg * trial elastic tangent
  int32_t shape;     // 0 quadratic B-spline, 1 cpGIMP (convected particle domain)
  int32_t pad_;
  double lp0[3];     // cpGIMP: initial half-width of the particle domain per axis
  int32_t elastic;   // 0 Hencky, 1 compressible Neo-Hookean (dp = 0 only)
  int32_t pad2_;
};

struct Particles {
  int64_t np;
  const double* x;     // [dim][np]
  const double* vol0;  // [np]
  const double* F;     // [dim*dim][np], row-major components
  const double* be;    // 2D [4][np] xx,yy,xy,zz ; 3D [6][np] xx,yy,zz,yz,xz,xy
  const double* fp;    // [dim][np] applied particle force or null
  const double* E;     // [np] or null
  const double* phi;   // [np] or null
};

inline int ndof_of(const Cfg& c) { return c.dim + (c.up ? 1 : 0); }
inline int64_t nodes_axis(const Cfg& c, int k) { return (int64_t)c.n[k] + 3; }
inline int64_t n_nodes(const Cfg& c) {
  int64_t t = 1; for (int k = 0; k < c.dim; ++k) t *= nodes_axis(c, k); return t; }
// linear index of node (i,j,k) with ghost shift (node -1 -> 0), x fastest
inline int64_t node_index(const Cfg& c, const int64_t* idx) {
  int64_t lin = 0, mult = 1;
  for (int k = 0; k < c.dim; ++k) { lin += (idx[k] + 1) * mult; mult *= nodes_axis(c, k); }
  return lin; }

// Per-particle state, promoted to scalar type T.
template <class T>
struct PState {
  T x[3];
  T vol0;
  M3<T> F, be;
  T E, phi;
  T fp[3];
};

template <class T>
PState<T> load_particle(const Cfg& c, const Particles& P, int64_t p) {
  PState<T> s;
  const int d = c.dim;
  const int64_t np = P.np;
  for (int k = 0; k < 3; ++k) { s.x[k] = T(0.0); s.fp[k] = T(0.0); }
  for (int k = 0; k < d; ++k) s.x[k] = T(P.x[k * np + p]);
  s.vol0 = T(P.vol0[p]);
  s.F = M3<T>::eye();
  for (int i = 0; i < d; ++i) for (int j = 0; j < d; ++j) s.F.a[i][j] = T(P.F[(i * d + j) * np + p]);
  s.be = M3<T>::eye();
  if (d == 2) {
    s.be.a[0][0] = T(P.be[0 * np + p]); s.be.a[1][1] = T(P.be[1 * np + p]);
    s.be.a[0][1] = s.be.a[1][0] = T(P.be[2 * np + p]); s.be.a[2][2] = T(P.be[3 * np + p]);
  } else {
    s.be.a[0][0] = T(P.be[0 * np + p]); s.be.a[1][1] = T(P.be[1 * np + p]); s.be.a[2][2] = T(P.be[2 * np + p]);
    s.be.a[1][2] = s.be.a[2][1] = T(P.be[3 * np + p]);
    s.be.a[0][2] = s.be.a[2][0] = T(P.be[4 * np + p]);
    s.be.a[0][1] = s.be.a[1][0] = T(P.be[5 * np + p]);
  }
  s.E = T(P.E ? P.E[p] : c.E);
  s.phi = T(P.phi ? P.phi[p] : c.phi);
  if (P.fp) for (int k = 0; k < d; ++k) s.fp[k] = T(P.fp[k * np + p]);
  return s;
}

// ------------------------------------------------------------- B-spline ----
// Quadratic B-spline, per axis.  u = (x - x0)/h; origin o = floor(u - 1/2);
// xi = u - o in [1/2, 3/2).  Node o+a sits at distance xi - a from the
// particle (in cells); N(r) = 3/4 - r^2 for |r| < 1/2, (3/2 - |r|)^2 / 2 for
// 1/2 <= |r| < 3/2.
template <class T>
void bspline_axis(const T& u, int64_t o, T w[3], T dwdu[3]) {
  T xi = u - (double)o;
  T r0 = 1.5 - xi, r1 = xi - 1.0, r2 = xi - 0.5;
  w[0] = 0.5 * r0 * r0;      dwdu[0] = -1.0 * r0;
  w[1] = 0.75 - r1 * r1;     dwdu[1] = -2.0 * r1;
  w[2] = 0.5 * r2 * r2;      dwdu[2] = 1.0 * r2;
}

inline int64_t origin_axis(double x, double x0, double h) { return (int64_t)std::floor((x - x0) / h - 0.5); }

// cpGIMP (Sec. 2.2 names the convected-particle-domain GIMP functions): the
// weight of a node is the average of its linear hat function over the
// particle's domain, a segment of half-width l (in cells) around the particle
// along each axis.  With r = particle minus node position (cells):
//   |r| < l          : 1 - (r^2 + l^2) / (2 l)
//   l <= |r| < 1 - l : 1 - |r|
//   1-l <= |r| < 1+l : (1 + l - |r|)^2 / (4 l)
//   otherwise        : 0
// For l <= 1/2 the nodes with a nonzero weight are o..o+2 of the B-spline
// origin o, so the stencil and the block pattern are the B-spline ones.
// dwdu is the derivative with respect to u = (x - x0)/h.
template <class T>
void gimp_axis(const T& u, int64_t o, const T& l, T w[3], T dwdu[3]) {
  for (int a = 0; a < 3; ++a) {
    T r = u - (double)(o + a);
    double rv = val(r), lv = val(l);
    double sg = rv < 0.0 ? -1.0 : 1.0;
    T ar = r * sg;
    if (std::fabs(rv) < lv) {
      w[a] = 1.0 - (r * r + l * l) / (2.0 * l);
      dwdu[a] = (-1.0) * r / l;
    } else if (std::fabs(rv) < 1.0 - lv) {
      w[a] = 1.0 - ar;
      dwdu[a] = T(-sg);
    } else if (std::fabs(rv) < 1.0 + lv) {
      T e = 1.0 + l - ar;
      w[a] = e * e / (4.0 * l);
      dwdu[a] = (-sg) * e / (2.0 * l);
    } else {
      w[a] = T(0.0);
      dwdu[a] = T(0.0);
    }
  }
}

template <class T>
struct Stencil {
  int nn;              // 3^d
  int64_t node[27];    // full-grid linear node indices
  T w[27];
  T grad[27][3];       // gradient w.r.t. x^n
};

template <class T>
Stencil<T> make_stencil(const Cfg& c, const PState<T>& s) {
  Stencil<T> st;
  const int d = c.dim;
  int64_t o[3] = {0, 0, 0};
  T w1[3][3], dw1[3][3];
  for (int k = 0; k < 3; ++k) for (int a = 0; a < 3; ++a) { w1[k][a] = T(1.0); dw1[k][a] = T(0.0); }
  for (int k = 0; k < d; ++k) {
    o[k] = origin_axis(val(s.x[k]), c.x0[k], c.h);
    T u = (s.x[k] - c.x0[k]) / c.h;
    if (c.shape == 1) {
      // the domain is convected with the stretch of its axis: l = lp0 F_kk
      T l = s.F.a[k][k] * (c.lp0[k] / c.h);
      gimp_axis(u, o[k], l, w1[k], dw1[k]);
    } else {
      bspline_axis(u, o[k], w1[k], dw1[k]);
    }
    for (int a = 0; a < 3; ++a) dw1[k][a] = dw1[k][a] / c.h;
  }
  st.nn = (d == 2) ? 9 : 27;
  for (int a = 0; a < st.nn; ++a) {
    int ia[3] = {a % 3, (a / 3) % 3, a / 9};
    int64_t idx[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) idx[k] = o[k] + ia[k];
    st.node[a] = node_index(c, idx);
    T wa = T(1.0);
    for (int k = 0; k < d; ++k) wa = wa * w1[k][ia[k]];
    st.w[a] = wa;
    for (int k = 0; k < 3; ++k) st.grad[a][k] = T(0.0);
    for (int k = 0; k < d; ++k) {
      T g = dw1[k][ia[k]];
      for (int m = 0; m < d; ++m) if (m != k) g = g * w1[m][ia[m]];
      st.grad[a][k] = g;
    }
  }
  return st;
}

// ------------------------------------------------------ constitutive -------
template <class T>
struct Moduli { T K, G, lam; };
template <class T>
Moduli<T> moduli(const T& E, double nu) {
  Moduli<T> m;
  m.K = E / (3.0 * (1.0 - 2.0 * nu));
  m.G = E / (2.0 * (1.0 + nu));
  m.lam = m.K - (2.0 / 3.0) * m.G;
  return m;
}

// Drucker-Prager coefficients: f = sqrt(J2) + eta p - xi c  (p = tr(tau)/3,
// tension positive); plastic potential g = sqrt(J2) + etabar p.
template <class T>
void dp_coeffs(int match, const T& phi, double psi, T& eta, T& xi, T& etabar) {
  const double r3 = std::sqrt(3.0);
  if (match == 3) {
    // J2 (von Mises) as the pressure-independent cone: sqrt(2 J2) <= c, i.e.
    // f = sqrt(J2) - c / sqrt(2) (Sec. 4.2, the elastoplastic bar); radial
    // return without volume change
    eta = T(0.0); xi = T(1.0 / std::sqrt(2.0)); etabar = T(0.0);
    (void)phi; (void)psi;
    return;
  }
  if (match == 1) {
    T t = tan(phi);
    T den = sqrt(9.0 + 12.0 * t * t);
    eta = 3.0 * t / den; xi = 3.0 / den;
    double tp = std::tan(psi);
    etabar = 3.0 * tp / std::sqrt(9.0 + 12.0 * tp * tp);
  } else if (match == 2) {
    T sp = sin(phi);
    eta = 6.0 * sp / (r3 * (3.0 + sp)); xi = 6.0 * cos(phi) / (r3 * (3.0 + sp));
    etabar = 6.0 * std::sin(psi) / (r3 * (3.0 + std::sin(psi)));
  } else {
    T sp = sin(phi);
    eta = 6.0 * sp / (r3 * (3.0 - sp)); xi = 6.0 * cos(phi) / (r3 * (3.0 - sp));
    etabar = 6.0 * std::sin(psi) / (r3 * (3.0 - std::sin(psi)));
  }
}

// Hencky + optional Drucker-Prager.  In: trial elastic log strain eps_tr.
// Out: Kirchhoff stress tau and the elastic log strain after return.
// Returns 0 elastic, 1 cone return, 2 apex return.
template <class T>
int hencky_dp(const Cfg& c, const T& E, const T& phi, const M3<T>& eps_tr, M3<T>& tau, M3<T>& eps_e) {
  Moduli<T> m = moduli(E, c.nu);
  T tr = trace(eps_tr);
  M3<T> tau_tr = scale(eps_tr, 2.0 * m.G);
  for (int i = 0; i < 3; ++i) tau_tr.a[i][i] += m.lam * tr;
  tau = tau_tr; eps_e = eps_tr;
  if (!c.dp) return 0;
  T eta, xi, etabar;
  dp_coeffs(c.dp_match & 3, phi, c.psi, eta, xi, etabar);
  if (c.dp_match & 4) etabar = eta;   // associated flow: the potential is the yield function
  T p = trace(tau_tr) / 3.0;
  M3<T> s = tau_tr;
  for (int i = 0; i < 3; ++i) s.a[i][i] -= p;
  double ss = 0; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) ss += val(s.a[i][j]) * val(s.a[i][j]);
  double q_val = std::sqrt(0.5 * ss);  // sqrt(J2), value only for the regime test
  double f_val = q_val + val(eta) * val(p) - val(xi) * c.c;
  if (f_val <= 0.0) return 0;
  // plastic: sqrt(J2) > 0 whenever the cone branch is taken (see below)
  T q = T(0.0);
  T f = T(0.0);
  if (q_val > 0.0) {
    T s2 = T(0.0);
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) s2 += s.a[i][j] * s.a[i][j];
    q = sqrt(0.5 * s2);
  }
  f = q + eta * p - xi * c.c;
  T dgam = f / (m.G + m.K * eta * etabar);
  T q_new = q - m.G * dgam;
  T p_new;
  M3<T> s_new;
  int regime;
  if (val(q_new) >= 0.0 && q_val > 0.0) {
    p_new = p - m.K * etabar * dgam;
    s_new = scale(s, q_new / q);
    regime = 1;
  } else {
    // apex: deviator vanishes, mean stress on the apex of the cone
    p_new = xi * c.c / eta;
    s_new = M3<T>::zero();
    regime = 2;
  }
  tau = s_new;
  for (int i = 0; i < 3; ++i) tau.a[i][i] += p_new;
  eps_e = scale(s_new, 1.0 / (2.0 * m.G));
  for (int i = 0; i < 3; ++i) eps_e.a[i][i] += p_new / (3.0 * m.K);
  if (regime == 2) {
    // The exact apex tangent of a cohesionless cone is zero, which leaves
    // nodes held only by apex particles without stiffness.  Derivatives (not
    // values) of an apex return are replaced by apex_reg times those of the
    // trial elastic stress; the residual is unchanged.
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) tau.a[i][j] = with_derivative(tau.a[i][j], tau_tr.a[i][j], c.apex_reg);
  }
  return regime;
}

// Kirchhoff stress from the trial left Cauchy-Green tensor b_tr.  Hencky
// (with the optional return map): eps_e receives the elastic log strain.
// Compressible Neo-Hookean (Sec. 4.5): tau = mu (b - 1) + lambda ln J 1 with
// J = sqrt(det b), b being the whole left Cauchy-Green tensor (no plasticity).
template <class T>
int stress_update(const Cfg& c, const T& E, const T& phi, const M3<T>& be_tr, M3<T>& tau, M3<T>& eps_e) {
  if (c.elastic == 1) {
    Moduli<T> m = moduli(E, c.nu);
    T lnJ = 0.5 * log(det(be_tr));
    tau = scale(sub(be_tr, M3<T>::eye()), m.G);
    for (int i = 0; i < 3; ++i) tau.a[i][i] += m.lam * lnJ;
    eps_e = M3<T>::zero();
    return 0;
  }
  M3<T> eps_tr = scale(logm_spd(be_tr), 0.5);
  return hencky_dp(c, E, phi, eps_tr, tau, eps_e);
}

// --------------------------------------------------- particle evaluation ---
// du_loc: local unknowns, node-interleaved [nn][ndof] (ndof = dim or dim+1).
// Outputs (each optional): fint_loc/fext_loc [nn][ndof]; new state.
template <class T>
int eval_particle(const Cfg& c, const PState<T>& s, const Stencil<T>& st, const T* du_loc,
                  T* fint_loc, T* fext_loc, PState<T>* snew) {
  const int d = c.dim, nd = ndof_of(c), nn = st.nn;
  // kinematics: dF = 1 + sum_a du_a (x) grad_a
  M3<T> dF = M3<T>::eye();
  for (int a = 0; a < nn; ++a)
    for (int i = 0; i < d; ++i) for (int j = 0; j < d; ++j) dF.a[i][j] += du_loc[a * nd + i] * st.grad[a][j];
  // trial state b_tr = dF b^e_n dF^T, then the stress
  M3<T> be_tr = mul(mul(dF, s.be), transpose(dF));
  M3<T> tau, eps_e;
  int regime = stress_update(c, s.E, s.phi, be_tr, tau, eps_e);
  M3<T> dFinvT = transpose(inverse(dF));
  T ddet = det(dF);
  T Jn = det(s.F);
  T J = ddet * Jn;
  T pp = T(0.0);
  T gp[3] = {T(0.0), T(0.0), T(0.0)};
  if (c.up) {
    for (int a = 0; a < nn; ++a) {
      pp += st.w[a] * du_loc[a * nd + d];
      for (int k = 0; k < d; ++k) gp[k] += st.grad[a][k] * du_loc[a * nd + d];
    }
    // total Kirchhoff stress: effective part minus b J p 1
    for (int i = 0; i < 3; ++i) tau.a[i][i] -= c.biot * J * pp;
  }
  M3<T> P = mul(tau, dFinvT);
  if (fint_loc) {
    for (int a = 0; a < nn; ++a) {
      for (int i = 0; i < d; ++i) {
        T f = T(0.0);
        for (int j = 0; j < d; ++j) f += P.a[i][j] * st.grad[a][j];
        fint_loc[a * nd + i] = s.vol0 * f;
      }
    }
    if (c.up) {
      // fluid mass balance (backward Euler, times dt):
      //   sum_p [ w b ln det(dF) + dt grad_x w . (k/mu)(grad_x p - rho_f g) ] J V0
      T gxp[3];
      for (int i = 0; i < 3; ++i) { gxp[i] = T(0.0); for (int j = 0; j < d; ++j) gxp[i] += dFinvT.a[i][j] * gp[j]; }
      T lnd = log(ddet);
      T mob = T(c.perm / c.mu_f);
      for (int a = 0; a < nn; ++a) {
        T flux = T(0.0);
        for (int i = 0; i < d; ++i) {
          T gxw = T(0.0);
          for (int j = 0; j < d; ++j) gxw += dFinvT.a[i][j] * st.grad[a][j];
          flux += gxw * (gxp[i] - c.rho_f * c.g[i]);
        }
        fint_loc[a * nd + d] = (st.w[a] * c.biot * lnd + c.dt * mob * flux) * J * s.vol0;
      }
    }
  }
  if (fext_loc) {
    for (int a = 0; a < nn; ++a) {
      for (int i = 0; i < d; ++i) fext_loc[a * nd + i] = st.w[a] * (c.rho0 * s.vol0 * c.g[i] + s.fp[i]);
      if (c.up) fext_loc[a * nd + d] = T(0.0);
    }
  }
  if (snew) {
    *snew = s;
    for (int i = 0; i < d; ++i) {
      T dx = T(0.0);
      for (int a = 0; a < nn; ++a) dx += st.w[a] * du_loc[a * nd + i];
      snew->x[i] = s.x[i] + dx;
    }
    snew->F = mul(dF, s.F);
    snew->be = c.elastic == 1 ? be_tr : expm_sym(scale(eps_e, 2.0));
  }
  return regime;
}

template <class T>
void store_state(const Cfg& c, const PState<T>& s, int64_t p, int64_t np, double* x, double* F, double* be) {
  const int d = c.dim;
  if (x) for (int k = 0; k < d; ++k) x[k * np + p] = val(s.x[k]);
  if (F) for (int i = 0; i < d; ++i) for (int j = 0; j < d; ++j) F[(i * d + j) * np + p] = val(s.F.a[i][j]);
  if (be) {
    if (d == 2) {
      be[0 * np + p] = val(s.be.a[0][0]); be[1 * np + p] = val(s.be.a[1][1]);
      be[2 * np + p] = val(s.be.a[0][1]); be[3 * np + p] = val(s.be.a[2][2]);
    } else {
      be[0 * np + p] = val(s.be.a[0][0]); be[1 * np + p] = val(s.be.a[1][1]); be[2 * np + p] = val(s.be.a[2][2]);
      be[3 * np + p] = val(s.be.a[1][2]); be[4 * np + p] = val(s.be.a[0][2]); be[5 * np + p] = val(s.be.a[0][1]);
    }
  }
}

template <class T>
void gather_local(const Cfg& c, const Stencil<T>& st, const double* dof_full, T* du_loc) {
  const int nd = ndof_of(c);
  for (int a = 0; a < st.nn; ++a)
    for (int k = 0; k < nd; ++k) du_loc[a * nd + k] = T(dof_full[st.node[a] * nd + k]);
}

// Local Jacobian of f_int for one particle via Dual<NL> seeded on its NL
// local unknowns.  K[r][c] = d fint_loc[r] / d du_loc[c].
template <int NL>
int local_jacobian(const Cfg& c, const Particles& P, int64_t p, const double* dof_full,
                   double* K, int64_t* nodes) {
  using D = Dual<NL>;
  PState<D> s = load_particle<D>(c, P, p);
  Stencil<D> st = make_stencil(c, s);
  D du[NL], fi[NL];
  gather_local(c, st, dof_full, du);
  for (int k = 0; k < NL; ++k) du[k].d[k] = 1.0;
  int reg = eval_particle(c, s, st, du, fi, (D*)nullptr, (PState<D>*)nullptr);
  for (int r = 0; r < NL; ++r) for (int q = 0; q < NL; ++q) K[r * NL + q] = fi[r].d[q];
  for (int a = 0; a < st.nn; ++a) nodes[a] = st.node[a];
  return reg;
}

// Particle state with forward tangents in two directions (for the
// sensitivity of a whole simulation to two material parameters).
struct Tangents {
  const double* x;      // [2][dim][np]
  const double* F;      // [2][dim*dim][np]
  const double* be;     // [2][nb][np]
  const double* theta;  // [2][2]: per direction, seeds of (E, phi)
};

inline PState<Dual<2>> load_particle_tan(const Cfg& c, const Particles& P, const Tangents& T, int64_t p) {
  using D = Dual<2>;
  PState<D> s = load_particle<D>(c, P, p);
  const int d = c.dim, nb = d == 2 ? 4 : 6;
  const int64_t np = P.np;
  for (int k = 0; k < 2; ++k) {
    for (int i = 0; i < d; ++i) s.x[i].d[k] = T.x[(k * d + i) * np + p];
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) s.F.a[i][j].d[k] = T.F[(k * d * d + i * d + j) * np + p];
    double b[6];
    for (int q = 0; q < nb; ++q) b[q] = T.be[(k * nb + q) * np + p];
    if (d == 2) {
      s.be.a[0][0].d[k] = b[0]; s.be.a[1][1].d[k] = b[1]; s.be.a[0][1].d[k] = s.be.a[1][0].d[k] = b[2];
      s.be.a[2][2].d[k] = b[3];
    } else {
      s.be.a[0][0].d[k] = b[0]; s.be.a[1][1].d[k] = b[1]; s.be.a[2][2].d[k] = b[2];
      s.be.a[1][2].d[k] = s.be.a[2][1].d[k] = b[3];
      s.be.a[0][2].d[k] = s.be.a[2][0].d[k] = b[4];
      s.be.a[0][1].d[k] = s.be.a[1][0].d[k] = b[5];
    }
    s.E.d[k] = T.theta[k * 2 + 0];
    s.phi.d[k] = T.theta[k * 2 + 1];
  }
  return s;
}

}  // namespace orc

using namespace orc;

// ======================================================== C interface =====
extern "C" {

// Internal and external nodal forces over the full padded grid (node-
// interleaved, ndof per node).  dof_full holds the unknowns (displacement
// increment, and nodal pore pressure for u-p).  regime (optional, [np])
// receives 0 elastic / 1 cone / 2 apex per particle.
int orc_forces(const Cfg* c, const Particles* P, const double* dof_full, double* fint, double* fext, int32_t* regime) {
  const int nd = ndof_of(*c);
  const int64_t nn_full = n_nodes(*c);
  const int64_t nv = nn_full * nd;
  std::memset(fint, 0, sizeof(double) * nv);
  if (fext) std::memset(fext, 0, sizeof(double) * nv);
  // particles split into one contiguous range per thread, each thread
  // scattering into its own full-grid copy; the copies are then summed in
  // thread order (the result depends on the thread count only through the
  // order of the sums)
  int nth = 1;
#ifdef _OPENMP
  nth = P->np >= 4096 ? omp_get_max_threads() : 1;
#endif
  std::vector<std::vector<double>> acc_i(nth), acc_e(nth);
#pragma omp parallel num_threads(nth)
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    std::vector<double>& ai = acc_i[t];
    std::vector<double>& ae = acc_e[t];
    ai.assign(nv, 0.0);
    if (fext) ae.assign(nv, 0.0);
    const int64_t p0 = P->np * t / nth, p1 = P->np * (t + 1) / nth;
    for (int64_t p = p0; p < p1; ++p) {
      PState<double> s = load_particle<double>(*c, *P, p);
      Stencil<double> st = make_stencil(*c, s);
      double du[27 * 4], fi[27 * 4], fe[27 * 4];
      gather_local(*c, st, dof_full, du);
      int reg = eval_particle(*c, s, st, du, fi, fe, (PState<double>*)nullptr);
      if (regime) regime[p] = reg;
      for (int a = 0; a < st.nn; ++a)
        for (int k = 0; k < nd; ++k) {
          ai[st.node[a] * nd + k] += fi[a * nd + k];
          if (fext) ae[st.node[a] * nd + k] += fe[a * nd + k];
        }
    }
  }
  for (int t = 0; t < nth; ++t) {
    for (int64_t i = 0; i < nv; ++i) fint[i] += acc_i[t][i];
    if (fext) for (int64_t i = 0; i < nv; ++i) fext[i] += acc_e[t][i];
  }
  return 0;
}

// Sum of weights * reference volume per node (full grid); a node with a zero
// sum carries no material even when it lies in a stencil.
int orc_node_volume(const Cfg* c, const Particles* P, double* out) {
  std::memset(out, 0, sizeof(double) * n_nodes(*c));
  for (int64_t p = 0; p < P->np; ++p) {
    PState<double> s = load_particle<double>(*c, *P, p);
    Stencil<double> st = make_stencil(*c, s);
    for (int a = 0; a < st.nn; ++a) out[st.node[a]] += st.w[a] * s.vol0;
  }
  return 0;
}

// Stencil origin per particle and axis: floor((x - x0)/h - 1/2)  ([dim][np]).
int orc_origins(const Cfg* c, const Particles* P, int64_t* o) {
  for (int64_t p = 0; p < P->np; ++p)
    for (int k = 0; k < c->dim; ++k) o[k * P->np + p] = origin_axis(P->x[k * P->np + p], c->x0[k], c->h);
  return 0;
}

static int local_jac_dispatch(const Cfg& c, const Particles& P, int64_t p, const double* dof, double* K, int64_t* nodes) {
  const int nl = (c.dim == 2 ? 9 : 27) * ndof_of(c);
  switch (nl) {
    case 18: return local_jacobian<18>(c, P, p, dof, K, nodes);
    case 27: return local_jacobian<27>(c, P, p, dof, K, nodes);
    case 81: return local_jacobian<81>(c, P, p, dof, K, nodes);
    case 108: return local_jacobian<108>(c, P, p, dof, K, nodes);
  }
  return -1;
}

// Local Jacobian blocks of every particle scattered into a caller-given BSR
// pattern (rows = active nodes, block size ndof, row-major blocks).
// row_of_node: full-grid node -> row index (or -1).  The caller zeroes val.
int orc_jacobian_bsr(const Cfg* c, const Particles* P, const double* dof_full, const int64_t* row_of_node,
                     const int32_t* rowptr, const int32_t* colind, double* val) {
  const int nd = ndof_of(*c);
  const int nn = (c->dim == 2) ? 9 : 27;
  const int nl = nn * nd;
  int err = 0;
#pragma omp parallel
  {
    std::vector<double> K(nl * nl);
    int64_t nodes[27];
#pragma omp for schedule(dynamic, 64)
    for (int64_t p = 0; p < P->np; ++p) {
      local_jac_dispatch(*c, *P, p, dof_full, K.data(), nodes);
      for (int a = 0; a < nn; ++a) {
        int64_t ra = row_of_node[nodes[a]];
        for (int b = 0; b < nn; ++b) {
          int64_t rb = row_of_node[nodes[b]];
          // locate column rb in row ra
          const int32_t* beg = colind + rowptr[ra];
          const int32_t* end = colind + rowptr[ra + 1];
          const int32_t* it = std::lower_bound(beg, end, (int32_t)rb);
          if (it == end || *it != rb) {
#pragma omp atomic write
            err = -1;
            continue;
          }
          int64_t blk = it - colind;
          for (int i = 0; i < nd; ++i)
            for (int j = 0; j < nd; ++j) {
              double v = K[(a * nd + i) * nl + (b * nd + j)];
#pragma omp atomic
              val[(blk * nd + i) * nd + j] += v;
            }
        }
      }
    }
  }
  return err;
}

// Dense Jacobian of f_int over ALL full-grid unknowns, one forward pass per
// seeded unknown (column by column).  out is [ntot][ntot] row-major where
// ntot = n_nodes * ndof.  Tiny grids only.
int orc_dense_jacobian(const Cfg* c, const Particles* P, const double* dof_full, double* out) {
  using D = Dual<1>;
  const int nd = ndof_of(*c);
  const int64_t ntot = n_nodes(*c) * nd;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t col = 0; col < ntot; ++col) {
    std::vector<double> colv(ntot, 0.0);
    for (int64_t p = 0; p < P->np; ++p) {
      PState<D> s = load_particle<D>(*c, *P, p);
      Stencil<D> st = make_stencil(*c, s);
      D du[27 * 4], fi[27 * 4];
      for (int a = 0; a < st.nn; ++a)
        for (int k = 0; k < nd; ++k) {
          int64_t gi = st.node[a] * nd + k;
          du[a * nd + k] = D(dof_full[gi]);
          if (gi == col) du[a * nd + k].d[0] = 1.0;
        }
      eval_particle(*c, s, st, du, fi, (D*)nullptr, (PState<D>*)nullptr);
      for (int a = 0; a < st.nn; ++a)
        for (int k = 0; k < nd; ++k) colv[st.node[a] * nd + k] += fi[a * nd + k].d[0];
    }
    for (int64_t r = 0; r < ntot; ++r) out[r * ntot + col] = colv[r];
  }
  return 0;
}

// End-of-step particle update: x += sum w du; F = dF F; b^e = exp(2 eps^e).
int orc_update(const Cfg* c, const Particles* P, const double* dof_full, double* x_out, double* F_out, double* be_out) {
  for (int64_t p = 0; p < P->np; ++p) {
    PState<double> s = load_particle<double>(*c, *P, p);
    Stencil<double> st = make_stencil(*c, s);
    double du[27 * 4];
    gather_local(*c, st, dof_full, du);
    PState<double> sn;
    eval_particle(*c, s, st, du, (double*)nullptr, (double*)nullptr, &sn);
    store_state(*c, sn, p, P->np, x_out, F_out, be_out);
  }
  return 0;
}

// Stress and regime per particle at the given unknowns: tau [9][np] (3x3
// Kirchhoff, row-major), regime [np].  Used by closed-form checks.
int orc_stress(const Cfg* c, const Particles* P, const double* dof_full, double* tau_out, int32_t* regime) {
  const int nd = ndof_of(*c);
  for (int64_t p = 0; p < P->np; ++p) {
    PState<double> s = load_particle<double>(*c, *P, p);
    Stencil<double> st = make_stencil(*c, s);
    double du[27 * 4];
    gather_local(*c, st, dof_full, du);
    M3<double> dF = M3<double>::eye();
    for (int a = 0; a < st.nn; ++a)
      for (int i = 0; i < c->dim; ++i) for (int j = 0; j < c->dim; ++j) dF.a[i][j] += du[a * nd + i] * st.grad[a][j];
    M3<double> be_tr = mul(mul(dF, s.be), transpose(dF));
    M3<double> tau, ee;
    int reg = stress_update(*c, s.E, s.phi, be_tr, tau, ee);
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) tau_out[(i * 3 + j) * P->np + p] = tau.a[i][j];
    if (regime) regime[p] = reg;
  }
  return 0;
}

// Forces and their tangents in two directions: the particle state carries
// tangents T, the unknowns carry dof_t ([2][n_nodes*ndof]).
// Outputs fint/fext (values) and fint_t/fext_t ([2][n_nodes*ndof]).
int orc_forces_tan(const Cfg* c, const Particles* P, const Tangents* T, const double* dof_full, const double* dof_t,
                   double* fint, double* fext, double* fint_t, double* fext_t) {
  using D = Dual<2>;
  const int nd = ndof_of(*c);
  const int64_t ntot = n_nodes(*c) * nd;
  std::memset(fint, 0, sizeof(double) * ntot);
  std::memset(fext, 0, sizeof(double) * ntot);
  std::memset(fint_t, 0, sizeof(double) * 2 * ntot);
  std::memset(fext_t, 0, sizeof(double) * 2 * ntot);
  for (int64_t p = 0; p < P->np; ++p) {
    PState<D> s = load_particle_tan(*c, *P, *T, p);
    Stencil<D> st = make_stencil(*c, s);
    D du[27 * 4], fi[27 * 4], fe[27 * 4];
    for (int a = 0; a < st.nn; ++a)
      for (int k = 0; k < nd; ++k) {
        int64_t gi = st.node[a] * nd + k;
        du[a * nd + k] = D(dof_full[gi]);
        du[a * nd + k].d[0] = dof_t[gi];
        du[a * nd + k].d[1] = dof_t[ntot + gi];
      }
    eval_particle(*c, s, st, du, fi, fe, (PState<D>*)nullptr);
    for (int a = 0; a < st.nn; ++a)
      for (int k = 0; k < nd; ++k) {
        int64_t gi = st.node[a] * nd + k;
        fint[gi] += fi[a * nd + k].v;
        fext[gi] += fe[a * nd + k].v;
        for (int q = 0; q < 2; ++q) {
          fint_t[q * ntot + gi] += fi[a * nd + k].d[q];
          fext_t[q * ntot + gi] += fe[a * nd + k].d[q];
        }
      }
  }
  return 0;
}

// End-of-step update with tangents: new state and its two tangent sets.
int orc_update_tan(const Cfg* c, const Particles* P, const Tangents* T, const double* dof_full, const double* dof_t,
                   double* x_out, double* F_out, double* be_out, double* x_t, double* F_t, double* be_t) {
  using D = Dual<2>;
  const int nd = ndof_of(*c), d = c->dim, nb = d == 2 ? 4 : 6;
  const int64_t ntot = n_nodes(*c) * nd, np = P->np;
  for (int64_t p = 0; p < np; ++p) {
    PState<D> s = load_particle_tan(*c, *P, *T, p);
    Stencil<D> st = make_stencil(*c, s);
    D du[27 * 4];
    for (int a = 0; a < st.nn; ++a)
      for (int k = 0; k < nd; ++k) {
        int64_t gi = st.node[a] * nd + k;
        du[a * nd + k] = D(dof_full[gi]);
        du[a * nd + k].d[0] = dof_t[gi];
        du[a * nd + k].d[1] = dof_t[ntot + gi];
      }
    PState<D> sn;
    eval_particle(*c, s, st, du, (D*)nullptr, (D*)nullptr, &sn);
    store_state(*c, sn, p, np, x_out, F_out, be_out);
    for (int q = 0; q < 2; ++q) {
      for (int i = 0; i < d; ++i) x_t[(q * d + i) * np + p] = sn.x[i].d[q];
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) F_t[(q * d * d + i * d + j) * np + p] = sn.F.a[i][j].d[q];
      double b[6];
      if (d == 2) {
        b[0] = sn.be.a[0][0].d[q]; b[1] = sn.be.a[1][1].d[q]; b[2] = sn.be.a[0][1].d[q]; b[3] = sn.be.a[2][2].d[q];
      } else {
        b[0] = sn.be.a[0][0].d[q]; b[1] = sn.be.a[1][1].d[q]; b[2] = sn.be.a[2][2].d[q];
        b[3] = sn.be.a[1][2].d[q]; b[4] = sn.be.a[0][2].d[q]; b[5] = sn.be.a[0][1].d[q];
      }
      for (int k = 0; k < nb; ++k) be_t[(q * nb + k) * np + p] = b[k];
    }
  }
  return 0;
}

// ---- standalone tensor functions, exposed for pins --------------------------
int orc_logm(const double* A, double* L) {
  M3<double> m; for (int i = 0; i < 9; ++i) m.a[i / 3][i % 3] = A[i];
  M3<double> r = logm_spd(m); for (int i = 0; i < 9; ++i) L[i] = r.a[i / 3][i % 3];
  return 0; }
int orc_expm(const double* A, double* E) {
  M3<double> m; for (int i = 0; i < 9; ++i) m.a[i / 3][i % 3] = A[i];
  M3<double> r = expm_sym(m); for (int i = 0; i < 9; ++i) E[i] = r.a[i / 3][i % 3];
  return 0; }
// Directional derivative of ln at A along dA (one dual direction).
int orc_logm_dir(const double* A, const double* dA, double* L, double* dL) {
  M3<Dual<1>> m;
  for (int i = 0; i < 9; ++i) { m.a[i / 3][i % 3] = Dual<1>(A[i]); m.a[i / 3][i % 3].d[0] = dA[i]; }
  M3<Dual<1>> r = logm_spd(m);
  for (int i = 0; i < 9; ++i) { L[i] = r.a[i / 3][i % 3].v; dL[i] = r.a[i / 3][i % 3].d[0]; }
  return 0; }
// Stress return for a given trial elastic log strain (3x3) and parameters.
int orc_return_map(const Cfg* c, double E, double phi, const double* eps_tr, double* tau, double* eps_e) {
  M3<double> e; for (int i = 0; i < 9; ++i) e.a[i / 3][i % 3] = eps_tr[i];
  M3<double> t, ee;
  int reg = hencky_dp(*c, E, phi, e, t, ee);
  for (int i = 0; i < 9; ++i) { tau[i] = t.a[i / 3][i % 3]; eps_e[i] = ee.a[i / 3][i % 3]; }
  return reg; }
// Directional derivative of the return map along d(eps_tr).
int orc_return_map_dir(const Cfg* c, double E, double phi, const double* eps_tr, const double* deps,
                       double* tau, double* dtau) {
  M3<Dual<1>> e;
  for (int i = 0; i < 9; ++i) { e.a[i / 3][i % 3] = Dual<1>(eps_tr[i]); e.a[i / 3][i % 3].d[0] = deps[i]; }
  M3<Dual<1>> t, ee;
  int reg = hencky_dp(*c, Dual<1>(E), Dual<1>(phi), e, t, ee);
  for (int i = 0; i < 9; ++i) { tau[i] = t.a[i / 3][i % 3].v; dtau[i] = t.a[i / 3][i % 3].d[0]; }
  return reg; }
int orc_gimp(double u, int64_t o, double l, double* w, double* dw) {
  gimp_axis<double>(u, o, l, w, dw);
  return 0;
}

int orc_bspline(double u, int64_t o, double* w, double* dw) {
  bspline_axis(u, o, w, dw); return 0; }

}  // extern "C"
