// Per (pixel, Gaussian) alpha bounds in FP32 with outward rounding (device code).
//
// Alg. GaussianSplat lines 9-10 as linear-relational operations (Sec. 3.3):
//   v = Add(Mul(d, d, u), -Mul(d, up))     v_k = u_k D2 - DUP_k       (exact scaling)
//   q = Mmul(v, Conic, Mp) = v B           q_n = Mul(v_0, B_0n) + Mul(v_1, B_1n)
//   s = Mmul(q, q^T)                       s = sum_n Sqr(q_n)
//   x = -s / 2,  a = o Exp(x)
// Every form is computed with round-to-nearest and its constant is then moved
// outward by a bound on the rounding error of the operation (magnitudes of the
// terms times a multiple of 2^-24), so each stored form bounds the true quantity.
// Concretised intervals are moved outward the same way.
#pragma once

#include <hip/hip_runtime.h>

#include "ar_internal.h"

namespace ar {

constexpr float kU = 0x1p-24f;  // unit roundoff of FP32

// s = q q^T bounds at one pixel; u = (ux, uy) centred pixel coordinates.
template <int P>
struct SForms {
  float sl[P + 1];  // lower form of s
  float sh[P + 1];  // upper form of s
  float slo, shi;   // interval of s (outward)
  float msl, msh;   // max over the box of |lower form|, |upper form|
};

template <int P>
__device__ __forceinline__ float abs_sum(const float *f) {
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < P; ++j) s += fabsf(f[j]);
  return s;
}

// (ux, uy): centred pixel coordinates as floats; (dux, duy) >= their distance to the
// exact coordinates (0 when the float is exact, as for half-integer principal points).
template <int P>
__device__ __forceinline__ void s_forms(const float *__restrict__ r, float ux, float uy, float dux, float duy,
                                        SForms<P> &o) {
  using R = Rec<P>;
  constexpr int F = P + 1;
  constexpr float KC = (P + 3) * kU;   // concretisation: P additions, one subtraction, the widening
  const float *sc = r + R::SC;

  // v_k = u_k * D2 - DUP_k on two-float operands: fma(u, hi, -hi') + fma(u, lo, -lo').
  // The first fma rounds the exact u*hi - hi' once, so the error is relative to v
  // itself: at most 2u|v| + 2u|second term| per coefficient, with the second term
  // below u (|u| M(D2) + M(DUP)).
  const float *d2l_h = r + R::D2, *d2l_l = d2l_h + F, *d2u_h = d2l_h + 2 * F, *d2u_l = d2l_h + 3 * F;
  float vl[2][F], vh[2][F], vlo[2], Mv[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float u = k ? uy : ux;
    const float *pl_h = r + R::DUP + 4 * F * k, *pl_l = pl_h + F, *pu_h = pl_h + 2 * F, *pu_l = pl_h + 3 * F;
    const bool pos = u >= 0.0f;
#pragma unroll
    for (int j = 0; j < F; ++j) {
      const float al_h = pos ? d2l_h[j] : d2u_h[j], al_l = pos ? d2l_l[j] : d2u_l[j];
      const float ah_h = pos ? d2u_h[j] : d2l_h[j], ah_l = pos ? d2u_l[j] : d2l_l[j];
      vl[k][j] = fmaf(u, al_h, -pu_h[j]) + fmaf(u, al_l, -pu_l[j]);
      vh[k][j] = fmaf(u, ah_h, -pl_h[j]) + fmaf(u, ah_l, -pl_l[j]);
    }
    float Sl = abs_sum<P>(vl[k]), Sh = abs_sum<P>(vh[k]);
    float Ml = fabsf(vl[k][P]) + Sl, Mh = fabsf(vh[k][P]) + Sh;
    const float du = k ? duy : dux;
    const float small = fmaf(du, sc[R::MD2], 4.0f * kU * kU * fmaf(fabsf(u), sc[R::MD2], sc[R::MDUP0 + k]));
    const float evl = fmaf(4.0f * kU, Ml, small), evh = fmaf(4.0f * kU, Mh, small);
    vl[k][P] -= evl;
    vh[k][P] += evh;
    Ml += evl;
    Mh += evh;
    vlo[k] = (vl[k][P] - Sl) - KC * Ml;
    Mv[k] = fmaxf(Ml, Mh);
  }

  // q_n = Mul(v_0, B_0n) + Mul(v_1, B_1n), McCormick with x = v (left operand):
  //   lower ylo*v_sel + vlo*B_sel - vlo*ylo, upper yhi*v_sel' + vlo*B_sel' - vlo*yhi
  // rounding: at most 6 roundings, each bounded by the magnitude sum Tq
  const float Tq = fmaf(sc[R::BMAX0], Mv[0],
                        fmaf(fabsf(vlo[0]), sc[R::MBB0], fmaf(sc[R::BMAX1], Mv[1], fabsf(vlo[1]) * sc[R::MBB1])));
  const float eq = 8.0f * kU * Tq;
#pragma unroll
  for (int j = 0; j < F; ++j) { o.sl[j] = 0.0f; o.sh[j] = 0.0f; }
  float es = 0.0f;
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    float ql[F], qh[F];
#pragma unroll
    for (int j = 0; j < F; ++j) { ql[j] = 0.0f; qh[j] = 0.0f; }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = 3 * k + n;
      const float *bl = r + R::B + 2 * F * e;
      const float *bh = bl + F;
      const float ylo = r[R::BI + e], yhi = r[R::BI + 6 + e];
      const bool yl_pos = ylo >= 0.0f, yh_pos = yhi >= 0.0f, vpos = vlo[k] >= 0.0f;
#pragma unroll
      for (int j = 0; j < F; ++j) {
        ql[j] = fmaf(ylo, yl_pos ? vl[k][j] : vh[k][j], fmaf(vlo[k], vpos ? bl[j] : bh[j], ql[j]));
        qh[j] = fmaf(yhi, yh_pos ? vh[k][j] : vl[k][j], fmaf(vlo[k], vpos ? bh[j] : bl[j], qh[j]));
      }
      ql[P] = fmaf(-vlo[k], ylo, ql[P]);
      qh[P] = fmaf(-vlo[k], yhi, qh[P]);
    }
    ql[P] -= eq;
    qh[P] += eq;
    const float Sl = abs_sum<P>(ql), Sh = abs_sum<P>(qh);
    const float Mlq = fabsf(ql[P]) + Sl, Mhq = fabsf(qh[P]) + Sh;
    const float qlo = (ql[P] - Sl) - KC * Mlq;
    const float qhi = (qh[P] + Sh) + KC * Mhq;
    const float Mq = fmaxf(Mlq, Mhq);
    // Sqr: tangent at xs = clamp(0, qlo, qhi) below, chord (qlo + qhi) q - qlo qhi above
    const float xs = fminf(fmaxf(qlo, 0.0f), qhi);
    const float t = xs + xs;
    const float m = qlo + qhi;
    const bool tpos = t >= 0.0f, mpos = m >= 0.0f;
#pragma unroll
    for (int j = 0; j < F; ++j) {
      o.sl[j] = fmaf(t, tpos ? ql[j] : qh[j], o.sl[j]);
      o.sh[j] = fmaf(m, mpos ? qh[j] : ql[j], o.sh[j]);
    }
    o.sl[P] = fmaf(-xs, xs, o.sl[P]);
    o.sh[P] = fmaf(-qlo, qhi, o.sh[P]);
    es = fmaf(Mq, Mq, es);
  }
  // each term of the three Sqr forms is at most 3 Mq^2 in magnitude; at most 9 roundings
  const float ees = 40.0f * kU * es;
  o.sl[P] -= ees;
  o.sh[P] += ees;
  const float Ssl = abs_sum<P>(o.sl), Ssh = abs_sum<P>(o.sh);
  o.msl = fabsf(o.sl[P]) + Ssl;
  o.msh = fabsf(o.sh[P]) + Ssh;
  o.slo = (o.sl[P] - Ssl) - KC * o.msl;
  o.shi = (o.sh[P] + Ssh) + KC * o.msh;
}

// Exp of x = -s/2 on [xlo, xhi] (Table "Bounds for operations Exp, Div and Ind"):
// tangent at xlo below, chord above, with the constants rounded outward.
struct ExpBounds {
  float xlo, xhi;
  float e_dn;   // <= exp(xlo): slope and value of the lower tangent
  float e_up;   // >= exp(xlo): anchor of the upper chord
  float k_up;   // >= chord slope over [xlo, xhi]
  float a_lo, a_hi;  // alpha interval o * [exp(xlo), exp(xhi)] outward
};

__device__ __forceinline__ void exp_bounds(float slo, float shi, float o, ExpBounds &b) {
  b.xlo = -0.5f * shi;
  b.xhi = -0.5f * fmaxf(slo, 0.0f);
  const float el = expf(b.xlo);
  const float eh = expf(b.xhi);
  b.e_dn = el * (1.0f - 4.0f * kU);
  b.e_up = el * (1.0f + 4.0f * kU);
  const float eh_up = eh * (1.0f + 4.0f * kU);
  const float dx = b.xhi - b.xlo;
  float k;
  if (dx < 0.5f) {
    k = dx > 0.0f ? el * (expm1f(dx) / dx) : el;
  } else {
    k = (eh_up - b.e_dn) / dx;
  }
  b.k_up = k * (1.0f + 16.0f * kU);
  b.a_lo = (o * b.e_dn) * (1.0f - 2.0f * kU);
  b.a_hi = fminf(o, (o * eh_up) * (1.0f + 2.0f * kU));
}

// Squared distance (float32, no contraction) from a pixel centre to the mean box; the
// pruning decision compares it with the record's r2.
__device__ __forceinline__ float dist2_box(float mu0lo, float mu0hi, float mu1lo, float mu1hi, float ux, float uy) {
#pragma clang fp contract(off)
  const float dx = fmaxf(fmaxf(mu0lo - ux, 0.0f), ux - mu0hi);
  const float dy = fmaxf(fmaxf(mu1lo - uy, 0.0f), uy - mu1hi);
  return dx * dx + dy * dy;
}

}  // namespace ar
