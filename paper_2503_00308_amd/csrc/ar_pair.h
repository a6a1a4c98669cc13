// Per (pixel, Gaussian) alpha bounds with outward rounding (device code).
//
// The q and a steps of Alg. GaussianSplat (Step 3) as linear-relational operations
// (Sec. 3.3):
//   v = Add(Mul(d, d, u), -Mul(d, up))     v_k = u_k D2 - DUP_k       (exact scaling)
//   q = Mmul(v, Conic, Mp) = v B           q_n = Mul(v_0, B_0n) + Mul(v_1, B_1n)
//   s = Mmul(q, q^T)                       s = sum_n Sqr(q_n)
//   x = -s / 2,  a = o Exp(x)
// All arithmetic is FP64 (on gfx950 an FP64 FMA issues at the rate of a non-packed
// FP32 one).  Form pairs are carried in mid-radius form (m, r): lower = m - r,
// upper = m + r.  Scaling by a of either sign gives (a m, |a| r), so the relaxations
// need no per-lane choice between the lower and the upper form.  Every operation is
// rounded to nearest; a bound on its rounding error (term magnitudes times small
// multiples of 2^-53) is added to the radius constant, and concretised intervals are
// moved outward the same way.
#pragma once

#include <hip/hip_runtime.h>

#include "ar_internal.h"
#include "ar_expm.h"

namespace ar {

constexpr double kU = 0x1p-53;    // unit roundoff of FP64
constexpr float kU32 = 0x1p-24f;  // unit roundoff of FP32

// Coefficients of the exp enclosure.  Pixel loops address the table at an offset that
// is zero at run time but depends on the Gaussian index (gid >> 31, gid < 2^31), so it
// is read through the scalar cache at every use instead of being kept in registers.
static __constant__ const double kExpTab[kExpTableLen] = AR_EXP_TABLE;

__device__ __forceinline__ const double *exp_table(uint32_t gid) { return kExpTab + (gid >> 31); }

// s = q q^T bounds at one pixel.
template <int P>
struct SForms {
  double sl[P + 1];  // lower form of s
  double sh[P + 1];  // upper form of s
  double slo, shi;   // interval of s (outward)
  double msl, msh;   // |constant| + sum |coefficients| of sl, sh
};

// (ux, uy): centred pixel coordinates (exact in FP64).
template <int P>
__device__ __forceinline__ void s_forms(const double *__restrict__ r, double ux, double uy, SForms<P> &o) {
  using R = Rec<P>;
  constexpr int F = P + 1;
  constexpr double KC = (P + 4) * kU;  // concretisation: P+1 additions, the subtractions, the widening

  // v_k = u_k D2 - DUP_k:  vm = u dm - pm,  vr = |u| dr + pr
  double vm[2][F], vr[2][F], vlo[2], Mv[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double u = k ? uy : ux;
    const double au = fabs(u);
    // product and sum rounded separately (both record values are uniform, and one FMA
    // may read only one of them from a scalar register)
    {
#pragma clang fp contract(off)
#pragma unroll
      for (int j = 0; j < F; ++j) {
        vm[k][j] = u * r[R::DM + j] - r[R::PM + F * k + j];
        vr[k][j] = au * r[R::DR + j] + r[R::PR + F * k + j];
      }
    }
    // sum_j |vm_j| + |vr_j| <= |u| MD2 + MDUP_k up to rounding; two roundings per
    // coefficient, each at most kU (|u| |dm_j| + |pm_j|) (resp. dr, pr)
    Mv[k] = fma(au, r[R::MD2], r[R::MDUP + k]) * (1.0 + 8.0 * kU);
    vr[k][P] += 2.0 * kU * Mv[k];
    double sl = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) sl += fabs(vm[k][j] - vr[k][j]);
    vlo[k] = ((vm[k][P] - vr[k][P]) - sl) - KC * Mv[k];
  }

  // q_n = sum_k Mul(v_k, B_kn), McCormick with x = v, y = B_kn in [ylo, yhi]:
  //   lower ylo v + vlo B - vlo ylo,  upper yhi v + vlo B - vlo yhi;  in mid-radius form
  //   qm = c1 vm + c2 vr + vlo Bm - vlo c1,   qr = c3 vm + c4 vr + |vlo| Br - vlo c3
  // with c1 = (ylo+yhi)/2, c2 = (|yhi|-|ylo|)/2, c3 = (yhi-ylo)/2, c4 = (|ylo|+|yhi|)/2.
  // The summed term magnitude over all coefficients is at most Tq; six roundings per
  // coefficient plus the rounding of the weights stay below 8 kU Tq.
  const double Tq = fma(2.0 * r[R::BMAX + 0], Mv[0],
                        fma(fabs(vlo[0]), r[R::MBB + 0],
                            fma(2.0 * r[R::BMAX + 1], Mv[1], fabs(vlo[1]) * r[R::MBB + 1])));
  const double eq = 8.0 * kU * Tq * (1.0 + 8.0 * kU);
#pragma unroll
  for (int j = 0; j < F; ++j) { o.sl[j] = 0.0; o.sh[j] = 0.0; }
  double es = 0.0;
#pragma unroll
  for (int n = 0; n < 3; ++n) {
    double qm[F], qr[F];
#pragma unroll
    for (int j = 0; j < F; ++j) { qm[j] = 0.0; qr[j] = 0.0; }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int e = 3 * k + n;
      const double *bm = r + R::BM + F * e;
      const double *br = r + R::BR + F * e;
      const double *cw = r + R::CM + 4 * e;
      const double a = vlo[k], aa = fabs(vlo[k]);
#pragma unroll
      for (int j = 0; j < F; ++j) {
        qm[j] = fma(cw[0], vm[k][j], fma(cw[1], vr[k][j], fma(a, bm[j], qm[j])));
        qr[j] = fma(cw[2], vm[k][j], fma(cw[3], vr[k][j], fma(aa, br[j], qr[j])));
      }
      qm[P] = fma(-a, cw[0], qm[P]);
      qr[P] = fma(-a, cw[2], qr[P]);
    }
    qr[P] += eq;
    // interval of q_n: lower form qm - qr, upper form qm + qr
    double Sl = 0.0, Sh = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      Sl += fabs(qm[j] - qr[j]);
      Sh += fabs(qm[j] + qr[j]);
    }
    const double qlc = qm[P] - qr[P], qhc = qm[P] + qr[P];
    const double Ml = fabs(qlc) + Sl, Mh = fabs(qhc) + Sh;
    const double wq = KC * (Ml + Mh);
    const double qlo = (qlc - Sl) - wq;
    const double qhi = (qhc + Sh) + wq;
    const double Mq = fmax(Ml, Mh) * (1.0 + 8.0 * kU);
    // Sqr: tangent at xs = clamp(0, qlo, qhi) below, chord (qlo + qhi) q - qlo qhi above
    //   lower  t qm - |t| qr - xs^2  (t = 2 xs),   upper  m qm + |m| qr - qlo qhi  (m = qlo + qhi)
    const double xs = fmin(fmax(qlo, 0.0), qhi);
    const double t = xs + xs, at = fabs(t);
    const double m = qlo + qhi, am = fabs(m);
#pragma unroll
    for (int j = 0; j < F; ++j) {
      o.sl[j] = fma(t, qm[j], fma(-at, qr[j], o.sl[j]));
      o.sh[j] = fma(m, qm[j], fma(am, qr[j], o.sh[j]));
    }
    o.sl[P] = fma(-xs, xs, o.sl[P]);
    o.sh[P] = fma(-qlo, qhi, o.sh[P]);
    es = fma(Mq, Mq, es);
  }
  // per n the Sqr terms sum to at most 10 Mq^2 over all coefficients; seven roundings each
  const double ees = 80.0 * kU * es;
  o.sl[P] -= ees;
  o.sh[P] += ees;
  double Ssl = 0.0, Ssh = 0.0;
#pragma unroll
  for (int j = 0; j < P; ++j) { Ssl += fabs(o.sl[j]); Ssh += fabs(o.sh[j]); }
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

// alpha interval [o_lo exp(xlo), o exp(xhi)] (o_lo = o for a plain scene)
__device__ __forceinline__ void exp_bounds(double slo, double shi, double o_lo, double o, ExpBounds &b,
                                           const double *cf) {
  b.xlo = -0.5 * shi;
  b.xhi = -0.5 * fmax(slo, 0.0);
  double eh_dn, eh_up, phi;
  const double h = b.xhi - b.xlo;
  exp_triple(b.xlo, b.xhi, h, b.e_dn, b.e_up, eh_dn, eh_up, phi, cf);
  double k;
  if (h <= 0.5) {
    // e^xlo (e^h - 1) / h; h is within u of the exact width, and the slope grows with h
    k = b.e_up * phi * (1.0 + 8.0 * kU);
  } else {
    k = (eh_up - b.e_dn) / h * (1.0 + 8.0 * kU);
  }
  b.k_up = k;
  b.a_lo = (o_lo * b.e_dn) * (1.0 - 2.0 * kU);
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
