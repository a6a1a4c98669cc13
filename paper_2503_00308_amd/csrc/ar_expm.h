// Rigorous FP64 enclosures of exp(x) and of (e^h - 1)/h, branch-light, for the Exp
// relaxation (Table "Bounds for operations Exp, Div and Ind").
//
// exp: Cody-Waite reduction x = k ln2 + r with ln2 split in a 42-bit head (k ln2_hi is
// exact for |k| < 2^11) and a tail, so |r| <= ln2/2 + 2^-50; then the degree-13 Taylor
// polynomial of e^r in Horner form and a scaling by 2^k.  Relative error budget for
// results >= 2^-1022 (x >= -708):
//   reduction       |r_computed - r| <= 2u|r| + 2^-80         -> < 2^-53
//   truncation      sum_{i>=14} |r|^i/i! <= |r|^14/14! e^|r|  -> < 2^-56 (|r| <= 0.3466)
//   coefficients    1/i! rounded to nearest                   -> <= u e^{2|r|} = 2u
//   Horner          13 fused steps, gamma_26 sum |c_i r^i|    -> <= 26u e^{2|r|} = 52u
// in total < 60u < 2^-47; the enclosure uses 2^-44.  Below x = -700 the enclosure is
// [0, 2^-1000] (e^-700 < 2^-1009).
//
// (e^h - 1)/h for 0 <= h <= 1/2: the Taylor series sum_n h^n/(n+1)!, degree 13;
// truncation h^14/15! / (1 - h/16) < 2^-54, Horner and coefficient rounding <= 27u of
// the value (which is >= 1); the enclosure uses 2^-44 as well.
//
// u = 2^-53.  AR_HD lets a host test compile the same functions.
#pragma once

#ifndef AR_HD
#define AR_HD __host__ __device__ __forceinline__
#endif

namespace ar {

constexpr double kExpRel = 0x1p-44;

// Coefficient table: 1/0! .. 1/14!, then log2(e), ln2 head, ln2 tail.
#define AR_EXP_TABLE                                                                         \
  {0x1p+0, 0x1p+0, 0x1p-1, 0x1.5555555555555p-3, 0x1.5555555555555p-5, 0x1.1111111111111p-7,   \
   0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19, \
   0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26, 0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33, \
   0x1.93974a8c07c9dp-37, 0x1.71547652b82fep+0, 0x1.62e42fefa3800p-1, 0x1.ef35793c76730p-45}
constexpr int kExpTableLen = 18;

// Horner evaluation of sum_{i=0..13} t^i / (i + s)!, s = 0 or 1 (c: the table above).
// The coefficients are positive; the |.| lets the GPU compiler take the addend straight
// from a scalar register instead of copying it into a vector register first.
template <int S>
AR_HD double taylor_exp_poly(double t, const double *c) {
  double p = c[13 + S];
#pragma unroll
  for (int i = 12; i >= 0; --i) p = fma(p, t, fabs(c[i + S]));
  return p;
}

// Cody-Waite reduction of x (clamped below at -745): x = kd ln2 + r
AR_HD double exp_reduce(double x, const double *c, double &kd) {
  const double xc = fmax(x, -745.0);
  kd = rint(xc * c[15]);                  // log2(e)
  const double r = fma(-kd, c[16], xc);   // ln2 head
  return fma(-kd, c[17], r);              // ln2 tail
}

AR_HD void exp_finish(double x, double p, double kd, double &dn, double &up) {
  const double e = ldexp(p, (int)kd);
  const bool tiny = x < -700.0;
  dn = tiny ? 0.0 : e * (1.0 - kExpRel);
  up = tiny ? 0x1p-1000 : e * (1.0 + kExpRel);
}

// dn <= exp(x) <= up for x <= 709
AR_HD void exp_encl(double x, double &dn, double &up, const double *c) {
  double kd;
  const double r = exp_reduce(x, c, kd);
  exp_finish(x, taylor_exp_poly<0>(r, c), kd, dn, up);
}

// an upper bound of (e^h - 1)/h for 0 <= h <= 1/2 (h = 0 gives 1)
AR_HD double expm1_over_x_up(double h, const double *c) {
  return taylor_exp_poly<1>(h, c) * (1.0 + kExpRel);
}

// The three enclosures the Exp relaxation needs, with the three Horner chains
// interleaved (each coefficient is read once): [d1, u1] of exp(x1), [d2, u2] of
// exp(x2), and phi >= (e^h - 1)/h (meaningful for 0 <= h <= 1/2).
AR_HD void exp_triple(double x1, double x2, double h, double &d1, double &u1, double &d2, double &u2, double &phi,
                      const double *c) {
  double k1, k2;
  const double r1 = exp_reduce(x1, c, k1);
  const double r2 = exp_reduce(x2, c, k2);
  double p1 = c[13], p2 = c[13], p3 = c[14];
#pragma unroll
  for (int i = 12; i >= 0; --i) {
    p1 = fma(p1, r1, fabs(c[i]));
    p2 = fma(p2, r2, fabs(c[i]));
    p3 = fma(p3, h, fabs(c[i + 1]));
  }
  exp_finish(x1, p1, k1, d1, u1);
  exp_finish(x2, p2, k2, d2, u2);
  phi = p3 * (1.0 + kExpRel);
}

}  // namespace ar
