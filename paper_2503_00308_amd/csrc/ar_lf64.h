// FP64 linear forms over the normalised pose box e in [-1,1]^P (device code).
//
// A quantity y is bounded by lower and upper affine forms,
//   lo[0..P) . e + lo[P] <= y(e) <= up[0..P) . e + up[P],
// the piecewise linear relations of Sec. 2.1.  The operations replace those of
// Alg. GaussianSplat by linear-relational ones (Sec. 3.3 item (2)):
//   Mul  McCormick planes through (xlo, ylo) (lower) and (xlo, yhi) (upper);
//   Sqr  tangent at the point of [xlo, xhi] closest to 0 (lower), chord (upper);
//   sin / cos of an exactly affine angle: Taylor-1 at the centre + Lagrange remainder.
#pragma once

#include <hip/hip_runtime.h>

namespace ar {

template <int P>
struct L64 {
  double lo[P + 1];
  double up[P + 1];
};

template <int P>
__host__ __device__ __forceinline__ L64<P> l_const(double c) {
  L64<P> r;
#pragma unroll
  for (int k = 0; k < P; ++k) { r.lo[k] = 0.0; r.up[k] = 0.0; }
  r.lo[P] = c;
  r.up[P] = c;
  return r;
}

// interval [min_e lower form, max_e upper form]
template <int P>
__host__ __device__ __forceinline__ void l_bounds(const L64<P> &x, double &lo, double &hi) {
  double sl = 0.0, sh = 0.0;
#pragma unroll
  for (int k = 0; k < P; ++k) { sl += fabs(x.lo[k]); sh += fabs(x.up[k]); }
  lo = x.lo[P] - sl;
  hi = x.up[P] + sh;
}

// max over the box of |form| (sum of |coefficients| and |constant|)
template <int P>
__host__ __device__ __forceinline__ double l_mag(const double *f) {
  double s = fabs(f[P]);
#pragma unroll
  for (int k = 0; k < P; ++k) s += fabs(f[k]);
  return s;
}

template <int P>
__host__ __device__ __forceinline__ L64<P> l_add(const L64<P> &a, const L64<P> &b) {
  L64<P> r;
#pragma unroll
  for (int k = 0; k <= P; ++k) { r.lo[k] = a.lo[k] + b.lo[k]; r.up[k] = a.up[k] + b.up[k]; }
  return r;
}

template <int P>
__host__ __device__ __forceinline__ L64<P> l_neg(const L64<P> &a) {
  L64<P> r;
#pragma unroll
  for (int k = 0; k <= P; ++k) { r.lo[k] = -a.up[k]; r.up[k] = -a.lo[k]; }
  return r;
}

template <int P>
__host__ __device__ __forceinline__ L64<P> l_sub(const L64<P> &a, const L64<P> &b) {
  return l_add<P>(a, l_neg<P>(b));
}

template <int P>
__host__ __device__ __forceinline__ L64<P> l_addc(const L64<P> &a, double c) {
  L64<P> r = a;
  r.lo[P] = a.lo[P] + c;
  r.up[P] = a.up[P] + c;
  return r;
}

// lower form of c*x for a constant c
template <int P>
__host__ __device__ __forceinline__ void l_scale_lower(const L64<P> &x, double c, double *out) {
  const double *f = c >= 0.0 ? x.lo : x.up;
#pragma unroll
  for (int k = 0; k <= P; ++k) out[k] = c * f[k];
}

template <int P>
__host__ __device__ __forceinline__ void l_scale_upper(const L64<P> &x, double c, double *out) {
  const double *f = c >= 0.0 ? x.up : x.lo;
#pragma unroll
  for (int k = 0; k <= P; ++k) out[k] = c * f[k];
}

template <int P>
__host__ __device__ __forceinline__ L64<P> l_scale(const L64<P> &x, double c) {
  L64<P> r;
  l_scale_lower<P>(x, c, r.lo);
  l_scale_upper<P>(x, c, r.up);
  return r;
}

// x * y, McCormick: lower ylo*x + xlo*y - xlo*ylo, upper yhi*x + xlo*y - xlo*yhi
template <int P>
__host__ __device__ __forceinline__ L64<P> l_mul(const L64<P> &x, const L64<P> &y) {
  double xlo, xhi, ylo, yhi;
  l_bounds<P>(x, xlo, xhi);
  l_bounds<P>(y, ylo, yhi);
  L64<P> r;
  double t[P + 1];
  l_scale_lower<P>(x, ylo, r.lo);
  l_scale_lower<P>(y, xlo, t);
#pragma unroll
  for (int k = 0; k <= P; ++k) r.lo[k] += t[k];
  l_scale_upper<P>(x, yhi, r.up);
  l_scale_upper<P>(y, xlo, t);
#pragma unroll
  for (int k = 0; k <= P; ++k) r.up[k] += t[k];
  r.lo[P] -= xlo * ylo;
  r.up[P] -= xlo * yhi;
  return r;
}

// x * x for one operand
template <int P>
__host__ __device__ __forceinline__ L64<P> l_sqr(const L64<P> &x) {
  double xlo, xhi;
  l_bounds<P>(x, xlo, xhi);
  const double xs = fmin(fmax(0.0, xlo), xhi);
  L64<P> r;
  l_scale_lower<P>(x, 2.0 * xs, r.lo);
  l_scale_upper<P>(x, xlo + xhi, r.up);
  r.lo[P] -= xs * xs;
  r.up[P] -= xlo * xhi;
  return r;
}

// sin (is_sin) or cos of an angle given as an exact affine form
template <int P>
__host__ __device__ __forceinline__ L64<P> l_trig(const L64<P> &th, bool is_sin) {
  const double c = th.lo[P];
  double rad = 0.0;
#pragma unroll
  for (int k = 0; k < P; ++k) rad += fabs(th.lo[k]);
  double s, co;
  sincos(c, &s, &co);
  const double f0 = is_sin ? s : co;
  const double f1 = is_sin ? co : -s;
  const double m2 = fmin(1.0, fabs(f0) + rad);
  const double rem = 0.5 * m2 * rad * rad;
  L64<P> r;
#pragma unroll
  for (int k = 0; k < P; ++k) { r.lo[k] = f1 * th.lo[k]; r.up[k] = f1 * th.lo[k]; }
  r.lo[P] = f0 - rem;
  r.up[P] = f0 + rem;
  return r;
}

}  // namespace ar
