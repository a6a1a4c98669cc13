// Per (pixel, Gaussian) alpha bounds with outward rounding (device code).
//
// Alg. GaussianSplat lines 9-10 as linear-relational operations (Sec. 3.3):
//   v = Add(Mul(d, d, u), -Mul(d, up))     v_k = u_k D2 - DUP_k       (exact scaling)
//   q = Mmul(v, Conic, Mp) = v B           q_n = Mul(v_0, B_0n) + Mul(v_1, B_1n)
//   s = Mmul(q, q^T)                       s = sum_n Sqr(q_n)
//   x = -s / 2,  a = o Exp(x)
// The forms are read from the FP32 record and evaluated in FP64: on gfx950 an FP64
// FMA issues at the rate of a non-packed FP32 one, and FP32 evaluation alone moved the
// upper image by several 1e-6 against the FP64 definition (coefficient roundings add up
// over the hundreds of Gaussians of a pixel's relational sum).  Every form is computed
// with round-to-nearest and its constant is then moved outward by a bound on the
// rounding error of the operation (term magnitudes times small multiples of 2^-53);
// concretised intervals are moved outward the same way.
#pragma once

#include <hip/hip_runtime.h>

#include "ar_internal.h"

namespace ar {

constexpr double kU = 0x1p-53;    // unit roundoff of FP64
constexpr float kU32 = 0x1p-24f;  // unit roundoff of FP32

// s = q q^T bounds at one pixel.
template <int P>
struct SForms {
  double sl[P + 1];  // lower form of s
  double sh[P + 1];  // upper form of s
  double slo, shi;   // interval of s (outward)
  double msl, msh;   // max over the box of |lower form|, |upper form|
};

template <int P>
__device__ __forceinline__ double abs_sum(const double *f) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < P; ++j) s += fabs(f[j]);
  return s;
}

// (ux, uy): centred pixel coordinates (FP64).
template <int P>
__device__ __forceinline__ void s_forms(const float *__restrict__ r, double ux, double uy, SForms<P> &o) {
  using R = Rec<P>;
  constexpr int F = P + 1;
  constexpr double KC = (P + 3) * kU;   // concretisation: P additions, one subtraction, the widening
  const float *sc = r + R::SC;

  // v_k = u_k * D2 - DUP_k; D2, DUP are two-float sums (exact in FP64): one fma each
  const float *d2l_h = r + R::D2, *d2l_l = d2l_h + F, *d2u_h = d2l_h + 2 * F, *d2u_l = d2l_h + 3 * F;
  double vl[2][F], vh[2][F], vlo[2], Mv[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double u = k ? uy : ux;
    const float *pl_h = r + R::DUP + 4 * F * k, *pl_l = pl_h + F, *pu_h = pl_h + 2 * F, *pu_l = pl_h + 3 * F;
    const bool pos = u >= 0.0;
#pragma unroll
    for (int j = 0; j < F; ++j) {
      const double dl = (double)d2l_h[j] + (double)d2l_l[j], du = (double)d2u_h[j] + (double)d2u_l[j];
      const double pl = (double)pl_h[j] + (double)pl_l[j], pu = (double)pu_h[j] + (double)pu_l[j];
      vl[k][j] = fma(u, pos ? dl : du, -pu);
      vh[k][j] = fma(u, pos ? du : dl, -pl);
    }
    // one rounding per coefficient, plus the rounding of u itself
    const double ev = 4.0 * kU * fma(fabs(u), (double)sc[R::MD2], (double)sc[R::MDUP0 + k]);
    vl[k][P] -= ev;
    vh[k][P] += ev;
    const double Sl = abs_sum<P>(vl[k]), Sh = abs_sum<P>(vh[k]);
    const double Ml = fabs(vl[k][P]) + Sl, Mh = fabs(vh[k][P]) + Sh;
    vlo[k] = (vl[k][P] - Sl) - KC * Ml;
    Mv[k] = fmax(Ml, Mh);
  }

  // q_n = Mul(v_0, B_0n) + Mul(v_1, B_1n), McCormick with x = v (left operand):
  //   lower ylo*v_sel + vlo*B_sel - vlo*ylo, upper yhi*v_sel' + vlo*B_sel' - vlo*yhi
  // at most 6 roundings, each bounded by the magnitude sum Tq
  const double Tq = fma((double)sc[R::BMAX0], Mv[0],
                        fma(fabs(vlo[0]), (double)sc[R::MBB0],
                            fma((double)sc[R::BMAX1], Mv[1], fabs(vlo[1]) * (double)sc[R::MBB1])));
  const double eq = 8.0 * kU * Tq;
#pragma unroll
  for (int j = 0; j < F; ++j) { o.sl[j] = 0.0; o.sh[j] = 0.0; }
  double es = 0.0;
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    double ql[F], qh[F];
#pragma unroll
    for (int j = 0; j < F; ++j) { ql[j] = 0.0; qh[j] = 0.0; }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = 3 * k + n;
      const float *bl = r + R::B + 2 * F * e;
      const float *bh = bl + F;
      const double ylo = (double)r[R::BI + e], yhi = (double)r[R::BI + 6 + e];
      const bool yl_pos = ylo >= 0.0, yh_pos = yhi >= 0.0, vpos = vlo[k] >= 0.0;
#pragma unroll
      for (int j = 0; j < F; ++j) {
        const double bsl = vpos ? (double)bl[j] : (double)bh[j];
        const double bsh = vpos ? (double)bh[j] : (double)bl[j];
        ql[j] = fma(ylo, yl_pos ? vl[k][j] : vh[k][j], fma(vlo[k], bsl, ql[j]));
        qh[j] = fma(yhi, yh_pos ? vh[k][j] : vl[k][j], fma(vlo[k], bsh, qh[j]));
      }
      ql[P] = fma(-vlo[k], ylo, ql[P]);
      qh[P] = fma(-vlo[k], yhi, qh[P]);
    }
    ql[P] -= eq;
    qh[P] += eq;
    const double Sl = abs_sum<P>(ql), Sh = abs_sum<P>(qh);
    const double Mlq = fabs(ql[P]) + Sl, Mhq = fabs(qh[P]) + Sh;
    const double qlo = (ql[P] - Sl) - KC * Mlq;
    const double qhi = (qh[P] + Sh) + KC * Mhq;
    const double Mq = fmax(Mlq, Mhq);
    // Sqr: tangent at xs = clamp(0, qlo, qhi) below, chord (qlo + qhi) q - qlo qhi above
    const double xs = fmin(fmax(qlo, 0.0), qhi);
    const double t = xs + xs;
    const double m = qlo + qhi;
    const bool tpos = t >= 0.0, mpos = m >= 0.0;
#pragma unroll
    for (int j = 0; j < F; ++j) {
      o.sl[j] = fma(t, tpos ? ql[j] : qh[j], o.sl[j]);
      o.sh[j] = fma(m, mpos ? qh[j] : ql[j], o.sh[j]);
    }
    o.sl[P] = fma(-xs, xs, o.sl[P]);
    o.sh[P] = fma(-qlo, qhi, o.sh[P]);
    es = fma(Mq, Mq, es);
  }
  // each term of the three Sqr forms is at most 3 Mq^2 in magnitude; at most 9 roundings
  const double ees = 40.0 * kU * es;
  o.sl[P] -= ees;
  o.sh[P] += ees;
  const double Ssl = abs_sum<P>(o.sl), Ssh = abs_sum<P>(o.sh);
  o.msl = fabs(o.sl[P]) + Ssl;
  o.msh = fabs(o.sh[P]) + Ssh;
  o.slo = (o.sl[P] - Ssl) - KC * o.msl;
  o.shi = (o.sh[P] + Ssh) + KC * o.msh;
}

// Exp of x = -s/2 on [xlo, xhi] (Table "Bounds for operations Exp, Div and Ind"):
// tangent at xlo below, chord above, with the constants rounded outward.
struct ExpBounds {
  double xlo, xhi;
  double e_dn;   // <= exp(xlo): slope and value of the lower tangent
  double e_up;   // >= exp(xlo): anchor of the upper chord
  double k_up;   // >= chord slope over [xlo, xhi]
  double a_lo, a_hi;  // alpha interval o * [exp(xlo), exp(xhi)] outward
};

__device__ __forceinline__ void exp_bounds(double slo, double shi, double o, ExpBounds &b) {
  b.xlo = -0.5 * shi;
  b.xhi = -0.5 * fmax(slo, 0.0);
  const double el = exp(b.xlo);
  const double eh = exp(b.xhi);
  b.e_dn = el * (1.0 - 4.0 * kU);
  b.e_up = el * (1.0 + 4.0 * kU);
  const double eh_up = eh * (1.0 + 4.0 * kU);
  const double dx = b.xhi - b.xlo;
  double k;
  if (dx < 0.5) {
    k = dx > 0.0 ? el * (expm1(dx) / dx) : el;
  } else {
    k = (eh_up - b.e_dn) / dx;
  }
  b.k_up = k * (1.0 + 16.0 * kU);
  b.a_lo = (o * b.e_dn) * (1.0 - 2.0 * kU);
  b.a_hi = fmin(o, (o * eh_up) * (1.0 + 2.0 * kU));
}

// Squared distance (float32, no contraction) from a pixel centre to the mean box; the
// pruning decision compares it with the record's r2.
__device__ __forceinline__ float dist2_box(float mu0lo, float mu0hi, float mu1lo, float mu1hi, float ux, float uy) {
#pragma clang fp contract(off)
  const float dx = fmaxf(fmaxf(mu0lo - ux, 0.0f), ux - mu0hi);
  const float dy = fmaxf(fmaxf(mu1lo - uy, 0.0f), uy - mu1hi);
  return dx * dx + dy * dy;
}

// Squared distance in FP64 from the exact pixel centre to the (float) mean box.
__device__ __forceinline__ double dist2_box64(const float *mu, double ux, double uy) {
  const double dx = fmax(fmax((double)mu[0] - ux, 0.0), ux - (double)mu[1]);
  const double dy = fmax(fmax((double)mu[2] - uy, 0.0), uy - (double)mu[3]);
  return dx * dx + dy * dy;
}

}  // namespace ar
