// Device-side mechanics for the implicit-MPM hot path (gfx950, FP64).
//
// Per particle: quadratic B-spline weights, the kinematics dF = 1 + du (x) grad w
// (Sec. 2.1), Hencky elasticity with a Drucker-Prager return map in
// Kirchhoff-stress / log-strain space, the first Piola-type stress
// P = tau dF^-T that the internal force f_int,i = V0 P grad w_i uses
// (Sec. 2.2: (grad^s w)^T : sigma V with sigma = tau / J and v = J V0), and
// the u-p terms (Sec. 2.2, Remark 1).
//
// Every routine is a template over the scalar S: S = double gives values,
// S = dnum carries one directional derivative, so the consistent tangent
// (the derivative of the stress update, Sec. 2.2) comes out of the same code
// by seeding one input per pass.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace mpm {

// ------------------------------------------------------------ dual number --
struct dnum {
  double v, d;
  dnum() = default;
  __host__ __device__ constexpr dnum(double x) : v(x), d(0.0) {}
  __host__ __device__ constexpr dnum(double x, double y) : v(x), d(y) {}
};
__device__ __forceinline__ dnum mk(double v, double d = 0.0) { return dnum{v, d}; }
__device__ __forceinline__ dnum operator+(dnum a, dnum b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ dnum operator-(dnum a, dnum b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ dnum operator-(dnum a) { return {-a.v, -a.d}; }
__device__ __forceinline__ dnum operator*(dnum a, dnum b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ dnum operator/(dnum a, dnum b) {
  double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ dnum operator+(dnum a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ dnum operator+(double b, dnum a) { return {a.v + b, a.d}; }
__device__ __forceinline__ dnum operator-(dnum a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ dnum operator-(double b, dnum a) { return {b - a.v, -a.d}; }
__device__ __forceinline__ dnum operator*(dnum a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ dnum operator*(double b, dnum a) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ dnum operator/(dnum a, double b) { return {a.v / b, a.d / b}; }
__device__ __forceinline__ dnum operator/(double a, dnum b) {
  double q = a / b.v;
  return {q, -q * b.d / b.v};
}
__device__ __forceinline__ dnum& operator+=(dnum& a, dnum b) { a.v += b.v; a.d += b.d; return a; }
__device__ __forceinline__ dnum& operator-=(dnum& a, dnum b) { a.v -= b.v; a.d -= b.d; return a; }

// value of a with the derivative of b scaled by f (plain values: a)
__device__ __forceinline__ double keep_value(double a, double, double) { return a; }
__device__ __forceinline__ dnum keep_value(dnum a, dnum b, double f) { return {a.v, f * b.d}; }

__device__ __forceinline__ double vv(double a) { return a; }
__device__ __forceinline__ double vv(dnum a) { return a.v; }
__device__ __forceinline__ double dd(dnum a) { return a.d; }

__device__ __forceinline__ double s_sqrt(double a) { return sqrt(a); }
__device__ __forceinline__ dnum s_sqrt(dnum a) { double r = sqrt(a.v); return {r, 0.5 * a.d / r}; }
__device__ __forceinline__ double s_log(double a) { return log(a); }
__device__ __forceinline__ dnum s_log(dnum a) { return {log(a.v), a.d / a.v}; }
__device__ __forceinline__ double s_exp(double a) { return exp(a); }
__device__ __forceinline__ dnum s_exp(dnum a) { double e = exp(a.v); return {e, e * a.d}; }
__device__ __forceinline__ double s_sin(double a) { return sin(a); }
__device__ __forceinline__ dnum s_sin(dnum a) { return {sin(a.v), cos(a.v) * a.d}; }
__device__ __forceinline__ double s_cos(double a) { return cos(a); }
__device__ __forceinline__ dnum s_cos(dnum a) { return {cos(a.v), -sin(a.v) * a.d}; }
__device__ __forceinline__ double s_tan(double a) { return tan(a); }
__device__ __forceinline__ dnum s_tan(dnum a) { double c = cos(a.v); return {tan(a.v), a.d / (c * c)}; }

// ------------------------------------------------------------- B-spline ----
// Quadratic B-spline along one axis.  u = (x - x0)/h, origin o = floor(u - 1/2),
// xi = u - o in [1/2, 3/2).  Node o+a is at signed distance xi - a (cells).
template <class S>
__device__ __forceinline__ void bspline3(S xi, double inv_h, S w[3], S dw[3]) {
  S r0 = 1.5 - xi, r1 = xi - 1.0, r2 = xi - 0.5;
  w[0] = 0.5 * r0 * r0;
  w[1] = 0.75 - r1 * r1;
  w[2] = 0.5 * r2 * r2;
  dw[0] = -1.0 * inv_h * r0;
  dw[1] = -2.0 * inv_h * r1;
  dw[2] = inv_h * r2;
}

// cpGIMP along one axis (Sec. 2.2): the weight of node o+a is the average of
// its linear hat function over the particle domain, half-width l cells
// (l <= 1/2), around the particle at signed distance r = xi - a from it:
//   |r| < l: 1 - (r^2 + l^2)/(2l);  l <= |r| < 1-l: 1 - |r|;
//   1-l <= |r| < 1+l: (1 + l - |r|)^2/(4l);  else 0.
__device__ __forceinline__ void gimp3(double xi, double l, double inv_h, double w[3], double dw[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double r = xi - a, ar = fabs(r), sg = r < 0.0 ? -1.0 : 1.0;
    double wa, da;
    if (ar < l) {
      wa = 1.0 - (r * r + l * l) / (2.0 * l);
      da = -r / l;
    } else if (ar < 1.0 - l) {
      wa = 1.0 - ar;
      da = -sg;
    } else if (ar < 1.0 + l) {
      const double e = 1.0 + l - ar;
      wa = e * e / (4.0 * l);
      da = -sg * e / (2.0 * l);
    } else {
      wa = 0.0;
      da = 0.0;
    }
    w[a] = wa;
    dw[a] = da * inv_h;
  }
}

// ---------------------------------------------------- material constants ---
template <class S>
struct Mat {
  S K, G, lam;          // bulk, shear, Lame lambda
  S eta, xi;            // cone slope and cohesion factor
  S etab;               // dilatancy slope of the plastic potential
  double c;             // cohesion
  double apex_reg;      // apex-return tangent scale
  int dp;
};

template <class S>
__device__ __forceinline__ Mat<S> make_mat(S E, double nu, S phi, double c, double psi, int dp, int match,
                                           double apex_reg) {
  Mat<S> m;
  m.apex_reg = apex_reg;
  m.K = E / (3.0 * (1.0 - 2.0 * nu));
  m.G = E / (2.0 * (1.0 + nu));
  m.lam = m.K - (2.0 / 3.0) * m.G;
  m.dp = dp;
  m.c = c;
  const double r3 = 1.7320508075688772935;
  const bool assoc = (match & 4) != 0;
  match &= 3;
  if (match == 3) {
    // J2: sqrt(2 J2) <= c, the pressure-independent cone (radial return)
    m.eta = S(0.0) * phi;
    m.xi = S(0.70710678118654752440) + 0.0 * phi;
    m.etab = S(0.0) * phi;
    return m;
  }
  if (match == 1) {
    S t = s_tan(phi);
    S den = s_sqrt(9.0 + 12.0 * t * t);
    m.eta = 3.0 * t / den;
    m.xi = 3.0 / den;
    double tp = tan(psi);
    m.etab = 3.0 * tp / sqrt(9.0 + 12.0 * tp * tp);
  } else {
    double sg = (match == 2) ? 1.0 : -1.0;   // 3 -+ sin(phi)
    S sp = s_sin(phi);
    S den = r3 * (3.0 + sg * sp);
    m.eta = 6.0 * sp / den;
    m.xi = 6.0 * s_cos(phi) / den;
    double spsi = sin(psi);
    m.etab = 6.0 * spsi / (r3 * (3.0 + sg * spsi));
  }
  if (assoc) m.etab = m.eta;   // associated flow: the potential is the yield function
  return m;
}

// ---------------------------------------------------------------- 2-D ------
// Plane strain: symmetric 3x3 tensors with zero xz, yz, stored as
// {xx, yy, xy, zz}.
template <class S>
struct Sym2 { S xx, yy, xy, zz; };

// atanh(t)/t as a function of t^2 (smooth at t = 0).
template <class S>
__device__ __forceinline__ S atanh_over(S t2) {
  if (vv(t2) < 1e-2) {
    // sum_k t^(2k)/(2k+1), k = 0..9  (truncation < 1e-20 for t^2 < 1e-2)
    S acc = S(1.0 / 19.0) + 0.0 * t2;
    acc = acc * t2 + 1.0 / 17.0; acc = acc * t2 + 1.0 / 15.0; acc = acc * t2 + 1.0 / 13.0;
    acc = acc * t2 + 1.0 / 11.0; acc = acc * t2 + 1.0 / 9.0;  acc = acc * t2 + 1.0 / 7.0;
    acc = acc * t2 + 1.0 / 5.0;  acc = acc * t2 + 1.0 / 3.0;  acc = acc * t2 + 1.0;
    return acc;
  }
  S t = s_sqrt(t2);
  return 0.5 * s_log((1.0 + t) / (1.0 - t)) / t;
}

// Hencky strain eps = 1/2 ln(b) of a plane-strain b (closed form: for a 2x2
// SPD block, ln A = 1/2 ln(det A) 1 + 2 atanh(t)/(t trA) (A - trA/2 1) with
// t^2 = ((a-c)^2 + 4 b^2)/(a+c)^2).
template <class S>
__device__ __forceinline__ Sym2<S> hencky2(const Sym2<S>& b) {
  S tr = b.xx + b.yy;
  S det = b.xx * b.yy - b.xy * b.xy;
  S df = b.xx - b.yy;
  S t2 = (df * df + 4.0 * b.xy * b.xy) / (tr * tr);
  S beta = atanh_over(t2) / tr;          // half of 2 atanh/(t tr)
  S hl = 0.25 * s_log(det);              // 1/2 * 1/2 ln det
  Sym2<S> e;
  e.xx = hl + 0.5 * beta * df;
  e.yy = hl - 0.5 * beta * df;
  e.xy = beta * b.xy;
  e.zz = 0.5 * s_log(b.zz);
  return e;
}

// b = exp(2 eps) for a plane-strain eps (closed form for the 2x2 block:
// exp A = e^m (cosh r 1 + sinh(r)/r (A - m 1)), m = trA/2, r^2 = ((a-c)/2)^2 + b^2).
template <class S>
__device__ __forceinline__ Sym2<S> exp2eps2(const Sym2<S>& e) {
  S a = 2.0 * e.xx, c = 2.0 * e.yy, b = 2.0 * e.xy;
  S m = 0.5 * (a + c);
  S hd = 0.5 * (a - c);
  S r2 = hd * hd + b * b;
  S ch, shr;   // cosh(r), sinh(r)/r as series in r^2 when small
  if (vv(r2) < 1e-2) {
    S c_acc = S(1.0 / 3628800.0) + 0.0 * r2, s_acc = S(1.0 / 39916800.0) + 0.0 * r2;
    const double cf[5] = {1.0 / 40320.0, 1.0 / 720.0, 1.0 / 24.0, 0.5, 1.0};
    const double sf[5] = {1.0 / 362880.0, 1.0 / 5040.0, 1.0 / 120.0, 1.0 / 6.0, 1.0};
    for (int k = 0; k < 5; ++k) { c_acc = c_acc * r2 + cf[k]; s_acc = s_acc * r2 + sf[k]; }
    ch = c_acc; shr = s_acc;
  } else {
    S r = s_sqrt(r2);
    S ep = s_exp(r), em = s_exp(-r);
    ch = 0.5 * (ep + em);
    shr = 0.5 * (ep - em) / r;
  }
  S em_ = s_exp(m);
  Sym2<S> out;
  out.xx = em_ * (ch + shr * hd);
  out.yy = em_ * (ch - shr * hd);
  out.xy = em_ * shr * b;
  out.zz = s_exp(2.0 * e.zz);
  return out;
}

// Hencky stress and Drucker-Prager return (perfect plasticity, tension
// positive, p = tr(tau)/3, f = sqrt(J2) + eta p - xi c, potential
// sqrt(J2) + etab p).  Returns 0 elastic, 1 cone, 2 apex.
// MS: the scalar type of the material constants (see stress3).
template <class S, class MS = S>
__device__ __forceinline__ int stress2(const Mat<MS>& m, const Sym2<S>& eps, Sym2<S>& tau, Sym2<S>& ee) {
  S trc = eps.xx + eps.yy + eps.zz;
  S lt = m.lam * trc;
  const MS g2 = 2.0 * m.G;
  tau.xx = lt + g2 * eps.xx; tau.yy = lt + g2 * eps.yy; tau.zz = lt + g2 * eps.zz; tau.xy = g2 * eps.xy;
  ee = eps;
  if (m.dp != 1) return 0;
  S p = (tau.xx + tau.yy + tau.zz) * (1.0 / 3.0);
  Sym2<S> s{tau.xx - p, tau.yy - p, tau.xy, tau.zz - p};
  double sv = vv(s.xx) * vv(s.xx) + vv(s.yy) * vv(s.yy) + vv(s.zz) * vv(s.zz) + 2.0 * vv(s.xy) * vv(s.xy);
  double qv = sqrt(0.5 * sv);
  double fv = qv + vv(m.eta) * vv(p) - vv(m.xi) * m.c;
  if (fv <= 0.0) return 0;
  int reg;
  S pn;
  if (qv > 0.0) {
    S q = s_sqrt(0.5 * (s.xx * s.xx + s.yy * s.yy + s.zz * s.zz + 2.0 * s.xy * s.xy));
    S f = q + m.eta * p - m.xi * m.c;
    S dg = f / (m.G + m.K * m.eta * m.etab);
    S qn = q - m.G * dg;
    if (vv(qn) >= 0.0) {
      S sc = qn / q;
      s.xx = s.xx * sc; s.yy = s.yy * sc; s.xy = s.xy * sc; s.zz = s.zz * sc;
      pn = p - m.K * m.etab * dg;
      reg = 1;
    } else {
      reg = 2;
    }
  } else {
    reg = 2;
  }
  if (reg == 2) {
    s.xx = s.xx * 0.0; s.yy = s.yy * 0.0; s.xy = s.xy * 0.0; s.zz = s.zz * 0.0;
    pn = m.xi * m.c / m.eta;
  }
  const Sym2<S> ttr = tau;
  tau.xx = s.xx + pn; tau.yy = s.yy + pn; tau.zz = s.zz + pn; tau.xy = s.xy;
  const MS i2g = 0.5 / m.G;
  const S i3k = pn / (3.0 * m.K);
  ee.xx = s.xx * i2g + i3k; ee.yy = s.yy * i2g + i3k; ee.zz = s.zz * i2g + i3k; ee.xy = s.xy * i2g;
  if (reg == 2) {
    // zero exact tangent at the apex of a cohesionless cone: keep the value,
    // take apex_reg times the trial elastic derivative
    tau.xx = keep_value(tau.xx, ttr.xx, m.apex_reg); tau.yy = keep_value(tau.yy, ttr.yy, m.apex_reg);
    tau.xy = keep_value(tau.xy, ttr.xy, m.apex_reg); tau.zz = keep_value(tau.zz, ttr.zz, m.apex_reg);
  }
  return reg;
}

// ---------------------------------------------------------------- 3-D ------
// Symmetric 3x3 stored as {xx, yy, zz, yz, xz, xy}.
template <class S>
struct Sym3 { S a[6]; };
template <class S>
__device__ __forceinline__ S sget(const Sym3<S>& A, int i, int j) {
  if (i == j) return A.a[i];
  int s = i + j;  // 1 -> xy(5), 2 -> xz(4), 3 -> yz(3)
  return A.a[s == 1 ? 5 : (s == 2 ? 4 : 3)];
}
// Product of two commuting symmetric matrices (result symmetric).
template <class S>
__device__ __forceinline__ Sym3<S> smul(const Sym3<S>& A, const Sym3<S>& B) {
  const int I[6] = {0, 1, 2, 1, 0, 0}, J[6] = {0, 1, 2, 2, 2, 1};
  Sym3<S> C;
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    C.a[t] = sget(A, I[t], 0) * sget(B, 0, J[t]) + sget(A, I[t], 1) * sget(B, 1, J[t]) +
             sget(A, I[t], 2) * sget(B, 2, J[t]);
  }
  return C;
}
template <class S>
__device__ __forceinline__ S sdet(const Sym3<S>& A) {
  return A.a[0] * (A.a[1] * A.a[2] - A.a[3] * A.a[3]) - A.a[5] * (A.a[5] * A.a[2] - A.a[3] * A.a[4]) +
         A.a[4] * (A.a[5] * A.a[3] - A.a[1] * A.a[4]);
}
template <class S>
__device__ __forceinline__ Sym3<S> sinv(const Sym3<S>& A) {
  Sym3<S> C;
  S d = sdet(A);
  S id = 1.0 / d;
  C.a[0] = (A.a[1] * A.a[2] - A.a[3] * A.a[3]) * id;
  C.a[1] = (A.a[0] * A.a[2] - A.a[4] * A.a[4]) * id;
  C.a[2] = (A.a[0] * A.a[1] - A.a[5] * A.a[5]) * id;
  C.a[3] = (A.a[4] * A.a[5] - A.a[0] * A.a[3]) * id;
  C.a[4] = (A.a[5] * A.a[3] - A.a[1] * A.a[4]) * id;
  C.a[5] = (A.a[3] * A.a[4] - A.a[2] * A.a[5]) * id;
  return C;
}
template <class S>
__device__ __forceinline__ double snorm_v(const Sym3<S>& A) {
  double s = 0;
#pragma unroll
  for (int t = 0; t < 6; ++t) s += (t < 3 ? 1.0 : 2.0) * vv(A.a[t]) * vv(A.a[t]);
  return sqrt(s);
}

// Hencky strain eps = 1/2 ln b of an SPD b.  b = c B with c = det(b)^(1/3),
// ln B = 2 atanh(Z) = 2 sum_{k odd} Z^k / k with Z = (B - 1)(B + 1)^-1.
// Sets *range_err when ||Z|| is beyond the series' working range.
template <class S>
__device__ __forceinline__ Sym3<S> hencky3(const Sym3<S>& b, int* range_err) {
  S ld = s_log(sdet(b));
  S cinv = s_exp(ld * (-1.0 / 3.0));
  Sym3<S> Bm, Bp;
#pragma unroll
  for (int t = 0; t < 6; ++t) { S v = b.a[t] * cinv; Bm.a[t] = v; Bp.a[t] = v; }
#pragma unroll
  for (int t = 0; t < 3; ++t) { Bm.a[t] = Bm.a[t] - 1.0; Bp.a[t] = Bp.a[t] + 1.0; }
  Sym3<S> Z = smul(Bm, sinv(Bp));
  double zn = snorm_v(Z);
  if (zn > 0.6) *range_err = 1;
  Sym3<S> Z2 = smul(Z, Z), term = Z, sum = Z;
  double tn = zn;
  for (int k = 3; k < 80; k += 2) {
    tn *= zn * zn;
    if (tn <= 1e-18 * zn * k || zn == 0.0) break;
    term = smul(term, Z2);
    double ik = 1.0 / k;
#pragma unroll
    for (int t = 0; t < 6; ++t) sum.a[t] = sum.a[t] + term.a[t] * ik;
  }
  Sym3<S> e;
  S third = ld * (1.0 / 6.0);   // 1/2 * (1/3) ln det
#pragma unroll
  for (int t = 0; t < 6; ++t) e.a[t] = sum.a[t];   // 1/2 * 2 * sum
#pragma unroll
  for (int t = 0; t < 3; ++t) e.a[t] = e.a[t] + third;
  return e;
}

// b = exp(2 eps): scaling and squaring around a Taylor series.
template <class S>
__device__ __forceinline__ Sym3<S> exp2eps3(const Sym3<S>& e) {
  Sym3<S> A;
#pragma unroll
  for (int t = 0; t < 6; ++t) A.a[t] = 2.0 * e.a[t];
  double n = snorm_v(A);
  int s = 0;
  while (n > 0.125 && s < 40) { n *= 0.5; ++s; }
  double sc = ldexp(1.0, -s);
#pragma unroll
  for (int t = 0; t < 6; ++t) A.a[t] = A.a[t] * sc;
  Sym3<S> sum, term;
#pragma unroll
  for (int t = 0; t < 6; ++t) { sum.a[t] = (t < 3 ? 1.0 : 0.0) + 0.0 * A.a[t]; term.a[t] = sum.a[t]; }
  for (int k = 1; k < 30; ++k) {
    term = smul(term, A);
    double ik = 1.0 / k;
#pragma unroll
    for (int t = 0; t < 6; ++t) { term.a[t] = term.a[t] * ik; sum.a[t] = sum.a[t] + term.a[t]; }
    if (snorm_v(term) < 1e-19) break;
  }
  for (int i = 0; i < s; ++i) sum = smul(sum, sum);
  return sum;
}

// MS: the scalar type of the material constants (plain double when only the
// state carries derivatives, as in the tangent tables; S when the
// derivatives with respect to E and the friction angle are wanted).
template <class S, class MS = S>
__device__ __forceinline__ int stress3(const Mat<MS>& m, const Sym3<S>& eps, Sym3<S>& tau, Sym3<S>& ee) {
  S trc = eps.a[0] + eps.a[1] + eps.a[2];
  S lt = m.lam * trc;
  const MS g2 = 2.0 * m.G;
#pragma unroll
  for (int t = 0; t < 6; ++t) tau.a[t] = g2 * eps.a[t];
#pragma unroll
  for (int t = 0; t < 3; ++t) tau.a[t] = tau.a[t] + lt;
  ee = eps;
  if (m.dp != 1) return 0;
  S p = (tau.a[0] + tau.a[1] + tau.a[2]) * (1.0 / 3.0);
  Sym3<S> s = tau;
#pragma unroll
  for (int t = 0; t < 3; ++t) s.a[t] = s.a[t] - p;
  double sv = 0;
#pragma unroll
  for (int t = 0; t < 6; ++t) sv += (t < 3 ? 1.0 : 2.0) * vv(s.a[t]) * vv(s.a[t]);
  double qv = sqrt(0.5 * sv);
  double fv = qv + vv(m.eta) * vv(p) - vv(m.xi) * m.c;
  if (fv <= 0.0) return 0;
  int reg = 2;
  S pn;
  if (qv > 0.0) {
    S ss = s.a[0] * s.a[0] + s.a[1] * s.a[1] + s.a[2] * s.a[2] +
           2.0 * (s.a[3] * s.a[3] + s.a[4] * s.a[4] + s.a[5] * s.a[5]);
    S q = s_sqrt(0.5 * ss);
    S f = q + m.eta * p - m.xi * m.c;
    S dg = f / (m.G + m.K * m.eta * m.etab);
    S qn = q - m.G * dg;
    if (vv(qn) >= 0.0) {
      S sc = qn / q;
#pragma unroll
      for (int t = 0; t < 6; ++t) s.a[t] = s.a[t] * sc;
      pn = p - m.K * m.etab * dg;
      reg = 1;
    }
  }
  if (reg == 2) {
#pragma unroll
    for (int t = 0; t < 6; ++t) s.a[t] = s.a[t] * 0.0;
    pn = m.xi * m.c / m.eta;
  }
  const MS i2g = 0.5 / m.G;
  const S i3k = pn / (3.0 * m.K);
  const Sym3<S> ttr = tau;
#pragma unroll
  for (int t = 0; t < 6; ++t) { tau.a[t] = s.a[t]; ee.a[t] = s.a[t] * i2g; }
#pragma unroll
  for (int t = 0; t < 3; ++t) { tau.a[t] = tau.a[t] + pn; ee.a[t] = ee.a[t] + i3k; }
  if (reg == 2)
#pragma unroll
    for (int t = 0; t < 6; ++t) tau.a[t] = keep_value(tau.a[t], ttr.a[t], m.apex_reg);
  return reg;
}

// ------------------------------------------------ particle stress output ---
// P = tau dF^-T per particle (the internal force is V0 P grad w), and the
// u-p terms of the fluid row.
struct UpPar { double biot, mob, dt, rho_f, g[3]; };


// -------------------------------------------------------- 2-D particle -----
template <class S>
struct Out2 { S P[2][2]; S s1; S vv[2]; };

template <class S, class MS = S>
__device__ __forceinline__ int mech2(const Mat<MS>& m, const S F[2][2], const Sym2<S>& be, S Jn, int up,
                                     const UpPar& u, S pp, const S gp[2], Out2<S>& o, Sym2<S>* be_out) {
  S m00 = F[0][0] * be.xx + F[0][1] * be.xy, m01 = F[0][0] * be.xy + F[0][1] * be.yy;
  S m10 = F[1][0] * be.xx + F[1][1] * be.xy, m11 = F[1][0] * be.xy + F[1][1] * be.yy;
  Sym2<S> bt;
  bt.xx = m00 * F[0][0] + m01 * F[0][1];
  bt.yy = m10 * F[1][0] + m11 * F[1][1];
  bt.xy = m00 * F[1][0] + m01 * F[1][1];
  bt.zz = be.zz;
  Sym2<S> tau, ee;
  int reg = 0;
  if (m.dp == 2) {
    // compressible Neo-Hookean: tau = mu (b - 1) + lambda ln J 1, J^2 = det b
    S lnJ = 0.5 * s_log((bt.xx * bt.yy - bt.xy * bt.xy) * bt.zz);
    S lj = m.lam * lnJ;
    tau.xx = m.G * (bt.xx - 1.0) + lj; tau.yy = m.G * (bt.yy - 1.0) + lj;
    tau.zz = m.G * (bt.zz - 1.0) + lj; tau.xy = m.G * bt.xy;
  } else {
    reg = stress2<S, MS>(m, hencky2(bt), tau, ee);
  }
  S det = F[0][0] * F[1][1] - F[0][1] * F[1][0];
  S idet = 1.0 / det;
  S it00 = F[1][1] * idet, it01 = -1.0 * F[1][0] * idet, it10 = -1.0 * F[0][1] * idet, it11 = F[0][0] * idet;
  S J = det * Jn;
  if (up) {
    S bp = u.biot * J * pp;
    tau.xx -= bp; tau.yy -= bp; tau.zz -= bp;
  }
  o.P[0][0] = tau.xx * it00 + tau.xy * it10;
  o.P[0][1] = tau.xx * it01 + tau.xy * it11;
  o.P[1][0] = tau.xy * it00 + tau.yy * it10;
  o.P[1][1] = tau.xy * it01 + tau.yy * it11;
  if (up) {
    o.s1 = u.biot * s_log(det) * J;
    S q0 = u.mob * (it00 * gp[0] + it01 * gp[1] - u.rho_f * u.g[0]);
    S q1 = u.mob * (it10 * gp[0] + it11 * gp[1] - u.rho_f * u.g[1]);
    o.vv[0] = u.dt * (it00 * q0 + it10 * q1) * J;
    o.vv[1] = u.dt * (it01 * q0 + it11 * q1) * J;
  }
  if (be_out) *be_out = (m.dp == 2) ? bt : exp2eps2(ee);   // b^e at the end of the step
  return reg;
}

// -------------------------------------------------------- 3-D particle -----
template <class S>
struct Out3 { S P[3][3]; };

template <class S, class MS = S>
__device__ __forceinline__ int mech3(const Mat<MS>& m, const S F[3][3], const Sym3<S>& be, Out3<S>& o,
                                     Sym3<S>* be_out, int* range_err) {
  S M[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[i][j] = F[i][0] * sget(be, 0, j) + F[i][1] * sget(be, 1, j) + F[i][2] * sget(be, 2, j);
  Sym3<S> bt;
  const int I[6] = {0, 1, 2, 1, 0, 0}, Jx[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
  for (int t = 0; t < 6; ++t)
    bt.a[t] = M[I[t]][0] * F[Jx[t]][0] + M[I[t]][1] * F[Jx[t]][1] + M[I[t]][2] * F[Jx[t]][2];
  Sym3<S> tau, ee;
  int reg = 0;
  if (m.dp == 2) {
    // compressible Neo-Hookean: tau = mu (b - 1) + lambda ln J 1, J^2 = det b
    S lj = m.lam * (0.5 * s_log(sdet(bt)));
#pragma unroll
    for (int t = 0; t < 6; ++t) tau.a[t] = m.G * bt.a[t];
#pragma unroll
    for (int t = 0; t < 3; ++t) tau.a[t] = tau.a[t] - m.G + lj;
  } else {
    reg = stress3<S, MS>(m, hencky3(bt, range_err), tau, ee);
  }
  // dF^-T = cofactor(dF) / det
  S cof[3][3];
  cof[0][0] = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  cof[0][1] = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  cof[0][2] = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  cof[1][0] = F[0][2] * F[2][1] - F[0][1] * F[2][2];
  cof[1][1] = F[0][0] * F[2][2] - F[0][2] * F[2][0];
  cof[1][2] = F[0][1] * F[2][0] - F[0][0] * F[2][1];
  cof[2][0] = F[0][1] * F[1][2] - F[0][2] * F[1][1];
  cof[2][1] = F[0][2] * F[1][0] - F[0][0] * F[1][2];
  cof[2][2] = F[0][0] * F[1][1] - F[0][1] * F[1][0];
  S det = F[0][0] * cof[0][0] + F[0][1] * cof[0][1] + F[0][2] * cof[0][2];
  S idet = 1.0 / det;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      o.P[i][j] = (sget(tau, i, 0) * cof[0][j] + sget(tau, i, 1) * cof[1][j] + sget(tau, i, 2) * cof[2][j]) * idet;
  if (be_out) *be_out = (m.dp == 2) ? bt : exp2eps3(ee);   // b^e at the end of the step
  return reg;
}

}  // namespace mpm
