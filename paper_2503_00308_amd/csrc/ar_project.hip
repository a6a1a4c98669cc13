// Pose stage and per-Gaussian stage of abstract rendering (FP64), gfx950.
//
// Pose stage (host and device): the set of cameras as linear forms
//   uc = A (uw - tau) + beta (the camera transform of Alg. GaussianSplat, Step 1, with R
//   and t replaced by their forms over the box).
// Per-Gaussian stage (one thread per Gaussian): Steps 1-2 of Alg. GaussianSplat and the
//   Conic of Step 3 as linear-relational operations (Sec. 3.3), MatrixInv for the
//   Conic (Sec. 3.1), and B = Conic * Mp hoisted out of the pixel loop (the q step
//   evaluated as v * (Conic Mp)).
//   The result is stored as an FP64 record of mid-radius form pairs, plus the
//   float32 footprint data used for pruning.
#include <hip/hip_runtime.h>
#include <math.h>

#include "ar_internal.h"
#include "ar_lf64.h"

namespace ar {

// ---------------------------------------------------------------------------------
// pose stage
// ---------------------------------------------------------------------------------
template <int P>
__host__ __device__ void store_form(double (*dst)[kMaxP + 1], const L64<P> &x) {
  for (int k = 0; k <= kMaxP; ++k) { dst[0][k] = 0.0; dst[1][k] = 0.0; }
  for (int k = 0; k < P; ++k) { dst[0][k] = x.lo[k]; dst[1][k] = x.up[k]; }
  dst[0][kMaxP] = x.lo[P];
  dst[1][kMaxP] = x.up[P];
}

template <int P>
__host__ __device__ __forceinline__ L64<P> load_form(const double (*src)[kMaxP + 1]) {
  L64<P> x;
#pragma unroll
  for (int k = 0; k < P; ++k) { x.lo[k] = src[0][k]; x.up[k] = src[1][k]; }
  x.lo[P] = src[0][kMaxP];
  x.up[P] = src[1][kMaxP];
  return x;
}

// elementary right-handed rotation (axis 0 = x, 1 = y, 2 = z) of an exact affine angle
template <int P>
__host__ __device__ void rot_forms(int axis, const L64<P> &ang, L64<P> R[9]) {
  const L64<P> c = l_trig<P>(ang, false);
  const L64<P> s = l_trig<P>(ang, true);
  const L64<P> ns = l_neg<P>(s);
  const L64<P> one = l_const<P>(1.0), zero = l_const<P>(0.0);
  if (axis == 0) {
    R[0] = one; R[1] = zero; R[2] = zero; R[3] = zero; R[4] = c; R[5] = ns; R[6] = zero; R[7] = s; R[8] = c;
  } else if (axis == 1) {
    R[0] = c; R[1] = zero; R[2] = s; R[3] = zero; R[4] = one; R[5] = zero; R[6] = ns; R[7] = zero; R[8] = c;
  } else {
    R[0] = c; R[1] = ns; R[2] = zero; R[3] = s; R[4] = c; R[5] = zero; R[6] = zero; R[7] = zero; R[8] = one;
  }
}

// C = Mmul(A, B) for 3x3 matrices of forms: C_ij = sum_t Mul(A_it, B_tj)
template <int P>
__host__ __device__ void mmul3(const L64<P> A[9], const L64<P> B[9], L64<P> C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      L64<P> acc = l_mul<P>(A[i * 3 + 0], B[0 * 3 + j]);
      acc = l_add<P>(acc, l_mul<P>(A[i * 3 + 1], B[1 * 3 + j]));
      acc = l_add<P>(acc, l_mul<P>(A[i * 3 + 2], B[2 * 3 + j]));
      C[i * 3 + j] = acc;
    }
}

template <int P>
__host__ __device__ L64<P> pose_param(const double *lo, const double *hi, int axis, const int *index) {
  const double c = 0.5 * (lo[axis] + hi[axis]);
  const double r = 0.5 * (hi[axis] - lo[axis]);
  L64<P> x = l_const<P>(c);
  if (index[axis] >= 0) {
    x.lo[index[axis]] = r;
    x.up[index[axis]] = r;
  }
  return x;
}

template <int P>
__host__ __device__ void pose_forms(const ar_pose_box &b, PoseForms &pf) {
  pf.P = P;
  L64<P> A[9], tau[3], beta[3];
  if (b.model == AR_POSE_CAMERA6) {
    int index[6];
    int p = 0;
    for (int a = 0; a < 6; ++a) index[a] = (b.hi[a] > b.lo[a]) ? p++ : -1;
    for (int k = 0; k < 3; ++k) tau[k] = l_addc<P>(pose_param<P>(b.lo, b.hi, k, index), b.t0[k]);
    L64<P> Ry[9], Rx[9], Rz[9], T1[9], T2[9], R0[9];
    rot_forms<P>(1, pose_param<P>(b.lo, b.hi, 3, index), Ry);
    rot_forms<P>(0, pose_param<P>(b.lo, b.hi, 4, index), Rx);
    rot_forms<P>(2, pose_param<P>(b.lo, b.hi, 5, index), Rz);
    for (int i = 0; i < 9; ++i) R0[i] = l_const<P>(b.R0[i]);
    mmul3<P>(Ry, Rx, T1);
    mmul3<P>(T1, Rz, T2);
    mmul3<P>(T2, R0, A);
    for (int k = 0; k < 3; ++k) beta[k] = l_const<P>(0.0);
  } else {
    int index[6] = {(b.hi[0] > b.lo[0]) ? 0 : -1, -1, -1, -1, -1, -1};
    L64<P> phi = pose_param<P>(b.lo, b.hi, 0, index);
    L64<P> Ry[9], R0[9];
    rot_forms<P>(1, l_neg<P>(phi), Ry);
    for (int i = 0; i < 9; ++i) R0[i] = l_const<P>(b.R0[i]);
    mmul3<P>(R0, Ry, A);
    for (int k = 0; k < 3; ++k) {
      tau[k] = l_const<P>(b.pivot[k]);
      double s = 0.0;
      for (int l = 0; l < 3; ++l) s += b.R0[k * 3 + l] * (b.pivot[l] - b.t0[l]);
      beta[k] = l_const<P>(s);
    }
  }
  for (int i = 0; i < 9; ++i) store_form<P>(pf.A[i], A[i]);
  for (int k = 0; k < 3; ++k) {
    store_form<P>(pf.tau[k], tau[k]);
    store_form<P>(pf.beta[k], beta[k]);
  }
  for (int l = 0; l < 3; ++l) {
    for (int k = 0; k <= kMaxP; ++k) {
      pf.Zm[l][k] = 0.5 * (pf.A[6 + l][0][k] + pf.A[6 + l][1][k]);
      pf.Zr[l][k] = 0.5 * (pf.A[6 + l][1][k] - pf.A[6 + l][0][k]);
    }
    // the lower and upper coefficients of a form need not be ordered, so a "radius"
    // Zr may be negative: magnitudes throughout; the sum's rounding (< 16 u of it) is far
    // inside the 2^-45 added
    double R = fabs(pf.Zr[l][kMaxP]);
    for (int k = 0; k < kMaxP; ++k) R += fabs(pf.Zm[l][k]) + fabs(pf.Zr[l][k]);
    pf.Zq[l] = R + 0x1p-45 * (fabs(pf.Zm[l][kMaxP]) + R);
  }
}

// ---------------------------------------------------------------------------------
// per-Gaussian stage
// ---------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t order_key(double d) {
  uint64_t b = __double_as_longlong(d);
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

// Store a (lower, upper) form pair in mid-radius form m = (l + h) / 2, r = (h - l) / 2.
// The radius constant absorbs the conversion rounding (at most 2^-53 of the summed
// magnitudes) and 2^-32 of the forms' magnitude, which covers the rounding of the FP64
// per-Gaussian stage.
template <int P>
__device__ __forceinline__ void store_mr(double *m, double *r, const L64<P> &x) {
  double mag = 0.0;
#pragma unroll
  for (int j = 0; j <= P; ++j) {
    m[j] = 0.5 * (x.lo[j] + x.up[j]);
    r[j] = 0.5 * (x.up[j] - x.lo[j]);
    mag += fabs(x.lo[j]) + fabs(x.up[j]);
  }
  r[P] += (0x1p-32 + 0x1p-50) * mag;
}

// sum_j |m_j| + |r_j| (>= the magnitude of both forms), rounded up
template <int P>
__device__ __forceinline__ double mag_mr(const double *m, const double *r) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j <= P; ++j) s += fabs(m[j]) + fabs(r[j]);
  return s * (1.0 + 0x1p-40);
}

// interval of a mid-radius form pair over the box, outward
template <int P>
__device__ __forceinline__ void bounds_mr(const double *m, const double *r, double &lo, double &hi) {
  double sl = 0.0, sh = 0.0;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    sl += fabs(m[j] - r[j]);
    sh += fabs(m[j] + r[j]);
  }
  const double w = 0x1p-40 * mag_mr<P>(m, r);
  lo = ((m[P] - r[P]) - sl) - w;
  hi = ((m[P] + r[P]) + sh) + w;
}

// The common start of MatrixInv (Sec. 3.1) for the symmetric 2x2 set
// X = [[x00, x01], [x01, x11]]: X0 the inverse of the interval-hull centre and
// IXX0 = I - X X0 (exact scaling of X's forms, widened by a bound on the FP64
// cancellation of the sum).  Returns false when the centre is not positive definite.
template <int P>
__device__ bool matinv_start(const L64<P> &x00, const L64<P> &x01, const L64<P> &x11, double X0[4], L64<P> E[4]) {
  double b00l, b00h, b01l, b01h, b11l, b11h;
  l_bounds<P>(x00, b00l, b00h);
  l_bounds<P>(x01, b01l, b01h);
  l_bounds<P>(x11, b11l, b11h);
  const double m00 = 0.5 * (b00l + b00h), m01 = 0.5 * (b01l + b01h), m11 = 0.5 * (b11l + b11h);
  const double det = m00 * m11 - m01 * m01;
  if (!(det > 0.0) || !isfinite(det)) return false;
  X0[0] = m11 / det;
  X0[1] = -m01 / det;
  X0[2] = -m01 / det;
  X0[3] = m00 / det;
  const L64<P> *X[4] = {&x00, &x01, &x01, &x11};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      L64<P> s = l_add<P>(l_scale<P>(*X[i * 2 + 0], X0[0 * 2 + j]), l_scale<P>(*X[i * 2 + 1], X0[1 * 2 + j]));
      L64<P> e = l_addc<P>(l_neg<P>(s), i == j ? 1.0 : 0.0);
      // cover the FP64 rounding of the cancelling sum I - X X0
      const double rho = 0x1p-50 * (l_mag<P>(X[i * 2 + 0]->lo) + l_mag<P>(X[i * 2 + 0]->up)) * fabs(X0[j]) +
                         0x1p-50 * (l_mag<P>(X[i * 2 + 1]->lo) + l_mag<P>(X[i * 2 + 1]->up)) * fabs(X0[2 + j]);
      e.lo[P] -= rho;
      e.up[P] += rho;
      E[i * 2 + j] = e;
    }
  return true;
}

// Eps = ||X0|| n^(k+1) / (1 - n) with n >= ||IXX0|| (Frobenius, from IXX0's intervals);
// false when the assertion n < 1 fails.
template <int P>
__device__ bool matinv_eps(const L64<P> E[4], const double X0[4], int k, double &eps) {
  double nn = 0.0;
  for (int i = 0; i < 4; ++i) {
    double lo, hi;
    l_bounds<P>(E[i], lo, hi);
    nn += fmax(lo * lo, hi * hi);
  }
  const double nbar = sqrt(nn);
  if (!(nbar < 1.0)) return false;
  const double nx0 = sqrt(X0[0] * X0[0] + X0[1] * X0[1] + X0[2] * X0[2] + X0[3] * X0[3]);
  eps = nx0 * pow(nbar, (double)(k + 1)) / (1.0 - nbar);
  return isfinite(eps);
}

// MatrixInv(X; X0, k) for the symmetric 2x2 set X = [[x00, x01], [x01, x11]] (Sec. 3.1):
//   IXX0 = I - X X0 with X0 the inverse of the interval-hull centre,
//   Xp = X0 sum_{i=0..k} IXX0^i,  Eps = ||X0|| n^(k+1) / (1 - n),  n >= ||IXX0||,
//   conic = <Xp - Eps, Xp + Eps>.  Returns false when the assertion n < 1 fails.
// Forward mode: every power carries its own pair of forms (l_mul).
template <int P>
__device__ bool matrix_inv(const L64<P> &x00, const L64<P> &x01, const L64<P> &x11, int k, L64<P> conic[4]) {
  double X0[4];
  L64<P> E[4];
  if (!matinv_start<P>(x00, x01, x11, X0, E)) return false;
  L64<P> S[4], Pw[4], T[4];
  for (int i = 0; i < 4; ++i) {
    S[i] = l_addc<P>(l_const<P>(0.0), (i == 0 || i == 3) ? 1.0 : 0.0);
    Pw[i] = E[i];
    S[i] = l_add<P>(S[i], E[i]);
  }
  for (int it = 2; it <= k; ++it) {
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        T[i * 2 + j] = l_add<P>(l_mul<P>(Pw[i * 2 + 0], E[0 * 2 + j]), l_mul<P>(Pw[i * 2 + 1], E[1 * 2 + j]));
    for (int i = 0; i < 4; ++i) {
      Pw[i] = T[i];
      S[i] = l_add<P>(S[i], T[i]);
    }
  }
  double eps;
  if (!matinv_eps<P>(E, X0, k, eps)) return false;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      L64<P> c = l_add<P>(l_scale<P>(S[0 * 2 + j], X0[i * 2 + 0]), l_scale<P>(S[1 * 2 + j], X0[i * 2 + 1]));
      c.lo[P] -= eps;
      c.up[P] += eps;
      conic[i * 2 + j] = c;
    }
  return true;
}

constexpr int kMaxTaylorK = 16;

// Backward substitution through MatrixInv's powers (Pw^1 = IXX0, Pw^i = Pw^(i-1) IXX0 by
// Mmul): an upper bound, as a form over e, of cst + sum over the levels L <= top of
// sum_ab D_ab Pw^L_ab (every level, or the top level only).  Each product
// Mul(Pw^(L-1)_at, IXX0_tb) is replaced by its McCormick plane (upper through (alo, bhi)
// for a positive weight, lower through (alo, blo) for a negative one, the left operand's
// lower bound alo taken from plo), so the weights flow to the level below and to IXX0;
// IXX0 = I - X X0 passes them on to the three inputs x00, x01 (both off-diagonal
// entries, one quantity) and x11, whose forms are substituted by the sign of their total
// weights.  The FP64 rounding of the substitution is covered by 2^-50 of its terms'
// magnitude, added to the constant.
template <int P>
__device__ void matinv_back(const L64<P> &x00, const L64<P> &x01, const L64<P> &x11, const double X0[4],
                            const double Elo[4], const double Ehi[4],
                            const double (*plo)[4], int top, const double D[4], bool every_level, double cst,
                            double out[P + 1]) {
  double W[4] = {0.0, 0.0, 0.0, 0.0}, V[4] = {0.0, 0.0, 0.0, 0.0};
  for (int lvl = top; lvl >= 2; --lvl) {
    double T[4];
    for (int q = 0; q < 4; ++q) {
      T[q] = (every_level || lvl == top) ? W[q] + D[q] : W[q];
      W[q] = 0.0;
    }
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const double w = T[a * 2 + b];
        if (w == 0.0) continue;
        for (int t = 0; t < 2; ++t) {
          const double alo = plo[lvl - 1][a * 2 + t];
          const double pe = w > 0.0 ? Ehi[t * 2 + b] : Elo[t * 2 + b];
          W[a * 2 + t] = fma(w, pe, W[a * 2 + t]);
          V[t * 2 + b] = fma(w, alo, V[t * 2 + b]);
          cst = fma(-w * alo, pe, cst);
        }
      }
  }
  for (int q = 0; q < 4; ++q) V[q] += (every_level || top == 1) ? W[q] + D[q] : W[q];
  // IXX0_ij = delta_ij - x_i0 X0_0j - x_i1 X0_1j, with x_10 = x_01
  const double U[3] = {-(V[0] * X0[0] + V[1] * X0[1]),
                       -(V[0] * X0[2] + V[1] * X0[3]) - (V[2] * X0[0] + V[3] * X0[1]),
                       -(V[2] * X0[2] + V[3] * X0[3])};
  cst += V[0] + V[3];
  const L64<P> *xs[3] = {&x00, &x01, &x11};
#pragma unroll
  for (int j = 0; j < P; ++j) out[j] = 0.0;
  out[P] = cst;
  double mag = fabs(cst);
  for (int q = 0; q < 3; ++q) {
    const double *f = U[q] > 0.0 ? xs[q]->up : xs[q]->lo;
#pragma unroll
    for (int j = 0; j <= P; ++j) out[j] = fma(U[q], f[j], out[j]);
    mag += fabs(U[q]) * l_mag<P>(f);
  }
  out[P] += 0x1p-50 * mag;
}

// MatrixInv with its linear bounds propagated backward (CROWN-style, the paper's bound
// engine): the same X0, IXX0, powers and Eps as matrix_inv, but every conic entry is
// bounded by one backward substitution from the entry to IXX0 (matinv_back), after the
// lower bounds of the powers' entries (the left operands of the next level's products)
// have been found the same way, level by level.
template <int P>
__device__ bool matrix_inv_backward(const L64<P> &x00, const L64<P> &x01, const L64<P> &x11, int k, L64<P> conic[4]) {
  double X0[4];
  L64<P> E[4];
  if (!matinv_start<P>(x00, x01, x11, X0, E)) return false;
  double eps;
  if (!matinv_eps<P>(E, X0, k, eps)) return false;
  double Elo[4], Ehi[4];
  for (int q = 0; q < 4; ++q) l_bounds<P>(E[q], Elo[q], Ehi[q]);
  double plo[kMaxTaylorK][4];
  for (int q = 0; q < 4; ++q) plo[1][q] = Elo[q];
  double f[P + 1];
  for (int lvl = 2; lvl < k; ++lvl)
    for (int q = 0; q < 4; ++q) {
      double D[4] = {0.0, 0.0, 0.0, 0.0};
      D[q] = -1.0;
      matinv_back<P>(x00, x01, x11, X0, Elo, Ehi, plo, lvl, D, false, 0.0, f);
      double s = f[P];
#pragma unroll
      for (int j = 0; j < P; ++j) s += fabs(f[j]);
      plo[lvl][q] = -s;
    }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      // conic_ij = sum_t X0_it S_tj, S = I + sum_L Pw^L
      double D[4] = {0.0, 0.0, 0.0, 0.0};
      for (int t = 0; t < 2; ++t) D[t * 2 + j] = X0[i * 2 + t];
      L64<P> c;
      matinv_back<P>(x00, x01, x11, X0, Elo, Ehi, plo, k, D, true, X0[i * 2 + j], c.up);
      for (int q = 0; q < 4; ++q) D[q] = -D[q];
      matinv_back<P>(x00, x01, x11, X0, Elo, Ehi, plo, k, D, true, -X0[i * 2 + j], c.lo);
#pragma unroll
      for (int t = 0; t <= P; ++t) c.lo[t] = -c.lo[t];
      c.lo[P] -= eps;
      c.up[P] += eps;
      conic[i * 2 + j] = c;
    }
  return true;
}

// The direct inverse that Sec. 3.1's Example 'matinv-vs-direct' compares MatrixInv with:
// adj(X) Div(det X), det = Mul(x00, x11) - Mul(x01, x01), Div as in Table "Bounds for
// operations Exp, Div and Ind" (tangent at the lower end below, chord above), entries
// Mul(adj_ij, 1/det).  Returns false where det is not provably positive.
template <int P>
__device__ bool adjugate_inv(const L64<P> &x00, const L64<P> &x01, const L64<P> &x11, L64<P> conic[4]) {
  const L64<P> det = l_sub<P>(l_mul<P>(x00, x11), l_mul<P>(x01, x01));
  double dlo, dhi;
  l_bounds<P>(det, dlo, dhi);
  if (!(dlo > 0.0) || !isfinite(dhi)) return false;
  L64<P> r;
  l_scale_lower<P>(det, -1.0 / (dlo * dlo), r.lo);
  l_scale_upper<P>(det, -1.0 / (dlo * dhi), r.up);
  r.lo[P] += 2.0 / dlo;
  r.up[P] += 1.0 / dlo + 1.0 / dhi;
  const L64<P> nx01 = l_neg<P>(x01);
  conic[0] = l_mul<P>(x11, r);
  conic[1] = l_mul<P>(nx01, r);
  conic[2] = l_mul<P>(nx01, r);
  conic[3] = l_mul<P>(x00, r);
  return true;
}

// Per-Gaussian stage of Gaussian g of the scene under pose forms `pose`; outputs at
// global index oi (cell * n + g when several cells are processed by one launch).
// CLASSIFY: only the Gaussian's type is decided, and counters points at its cell's two
// counts (MatrixInv failures the pruning test keeps somewhere in the image, near-plane
// straddlers); nothing else is written.
template <int P, bool CLASSIFY = false>
__device__ __forceinline__ void project_one(const SceneDev &sc, const PoseForms &pose, const Params &prm, int g,
                                            size_t oi, double *__restrict__ rec_out, uint64_t *__restrict__ key_out,
                                            uint64_t *__restrict__ key_sort, uint32_t *__restrict__ perm_out,
                                            int32_t *__restrict__ rect_out, double *__restrict__ dform_out,
                                            double *__restrict__ dint_out, unsigned long long *__restrict__ counters,
                                            double eps_cull) {
  const int n = sc.n;
  double uw[3] = {sc.mean[g], sc.mean[n + g], sc.mean[2 * n + g]};
  // a set of scenes (Sec. 4.6): the mean moved by scene variable v, uw + dir s_v, is the
  // form uw + dir (s_mid + s_rad e_(pose_vars + v)); uw holds its centre below
  const int mv = sc.mean_var ? sc.mean_var[g] : -1;
  double mdir[3] = {0.0, 0.0, 0.0};
  if (mv >= 0) {
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      mdir[l] = sc.mean_dir[(size_t)l * n + g];
      uw[l] += mdir[l] * sc.s_mid[mv];
    }
  }
  double Mw[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Mw[i] = sc.cov[(size_t)i * n + g];
  const float o = sc.opac[g];
  if constexpr (!CLASSIFY) perm_out[oi] = (uint32_t)oi;

  // Step 1: uc = Mmul(A, Add(uw, -tau)) + beta
  L64<P> y[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) y[l] = l_addc<P>(l_neg<P>(load_form<P>(pose.tau[l])), uw[l]);
  if (mv >= 0) {
    const int ix = prm.pose_vars + mv;   // < P (checked on the host)
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int k = 0; k < P; ++k)
        if (k == ix) {
          y[l].lo[k] += mdir[l] * sc.s_rad[mv];
          y[l].up[k] += mdir[l] * sc.s_rad[mv];
        }
  }
  L64<P> uc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    L64<P> acc = l_mul<P>(load_form<P>(pose.A[k * 3 + 0]), y[0]);
    acc = l_add<P>(acc, l_mul<P>(load_form<P>(pose.A[k * 3 + 1]), y[1]));
    acc = l_add<P>(acc, l_mul<P>(load_form<P>(pose.A[k * 3 + 2]), y[2]));
    uc[k] = l_add<P>(acc, load_form<P>(pose.beta[k]));
  }
  const L64<P> &x = uc[0], &yy = uc[1], &d = uc[2];   // Step 2: d = uc_z
  const double fx = prm.fx, fy = prm.fy;
  // Step 2: J (its non-zero entries) and up with the principal point removed
  const L64<P> J00 = l_scale<P>(d, fx), J02 = l_scale<P>(x, -fx);
  const L64<P> J11 = l_scale<P>(d, fy), J12 = l_scale<P>(yy, -fy);
  const L64<P> up0 = l_scale<P>(x, fx), up1 = l_scale<P>(yy, fy);
  // Steps 1-2: Mc = Mmul(A, Mw) (Mw constant), Mp = Mmul(J, Mc)
  L64<P> Mp0[3], Mp1[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    L64<P> Mc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      L64<P> acc = l_scale<P>(load_form<P>(pose.A[k * 3 + 0]), Mw[0 * 3 + m]);
      acc = l_add<P>(acc, l_scale<P>(load_form<P>(pose.A[k * 3 + 1]), Mw[1 * 3 + m]));
      acc = l_add<P>(acc, l_scale<P>(load_form<P>(pose.A[k * 3 + 2]), Mw[2 * 3 + m]));
      Mc[k] = acc;
    }
    Mp0[m] = l_add<P>(l_mul<P>(J00, Mc[0]), l_mul<P>(J02, Mc[2]));
    Mp1[m] = l_add<P>(l_mul<P>(J11, Mc[1]), l_mul<P>(J12, Mc[2]));
  }
  // factors of the q step: d*d and d*up
  const L64<P> D2 = l_sqr<P>(d);
  const L64<P> DUP0 = l_mul<P>(d, up0), DUP1 = l_mul<P>(d, up1);
  // Step 3, Conic: X = Mmul(Mp, Mp^T)
  L64<P> X00 = l_sqr<P>(Mp0[0]), X11 = l_sqr<P>(Mp1[0]), X01 = l_mul<P>(Mp0[0], Mp1[0]);
#pragma unroll
  for (int m = 1; m < 3; ++m) {
    X00 = l_add<P>(X00, l_sqr<P>(Mp0[m]));
    X11 = l_add<P>(X11, l_sqr<P>(Mp1[m]));
    X01 = l_add<P>(X01, l_mul<P>(Mp0[m], Mp1[m]));
  }

  // near plane and footprint
  double dlo, dhi;
  l_bounds<P>(d, dlo, dhi);
  const bool dropped = dhi <= prm.z_near;
  const bool straddle = !dropped && dlo <= prm.z_near;
  double u0lo, u0hi, u1lo, u1hi;
  l_bounds<P>(up0, u0lo, u0hi);
  l_bounds<P>(up1, u1lo, u1hi);
  double alo, ahi, blo, bhi, clo, chi;
  l_bounds<P>(X00, alo, ahi);
  l_bounds<P>(X01, blo, bhi);
  l_bounds<P>(X11, clo, chi);
  double m0lo = 0, m0hi = 0, m1lo = 0, m1hi = 0, lam = 0, r2 = -1;
  bool geo_ok = false;
  if (dlo > 0.0) {
    m0lo = fmin(u0lo / dlo, u0lo / dhi);
    m0hi = fmax(u0hi / dlo, u0hi / dhi);
    m1lo = fmin(u1lo / dlo, u1lo / dhi);
    m1hi = fmax(u1hi / dlo, u1hi / dhi);
    const double lamx = 0.5 * (ahi + chi) +
                        sqrt(0.25 * fmax((ahi - clo) * (ahi - clo), (chi - alo) * (chi - alo)) + fmax(blo * blo, bhi * bhi));
    const double dl2 = dlo * dlo;
    lam = lamx / (dl2 * dl2);
    r2 = ((double)o > eps_cull) ? 2.0 * lam * log((double)o / eps_cull) : -1.0;
    geo_ok = isfinite(m0lo) && isfinite(m0hi) && isfinite(m1lo) && isfinite(m1hi) && isfinite(lam) &&
             isfinite(r2) && lam > 0.0;
  }
  const bool normal = !dropped && !straddle && geo_ok;
  int32_t type = dropped ? kDropped : (normal ? kNormal : kWild);

  L64<P> conic[4];
  if (normal) {
    const bool inv_ok = prm.inverse == 1 ? matrix_inv_backward<P>(X00, X01, X11, prm.taylor_k, conic)
                        : prm.inverse == 2 ? adjugate_inv<P>(X00, X01, X11, conic)
                                           : matrix_inv<P>(X00, X01, X11, prm.taylor_k, conic);
    if (!inv_ok) type = kFallback;
  }
  if constexpr (CLASSIFY) {
    if (type == kFallback) {
      // kept at some pixel: the binning's float32 test on the rectangle of all pixel centres
      const float mu[4] = {__double2float_rd(m0lo), __double2float_ru(m0hi), __double2float_rd(m1lo),
                           __double2float_ru(m1hi)};
      const float ux0 = (float)(0.5 - prm.cx), ux1 = (float)((double)(prm.width - 1) + 0.5 - prm.cx);
      const float uy0 = (float)(0.5 - prm.cy), uy1 = (float)((double)(prm.height - 1) + 0.5 - prm.cy);
      if (dist2_rect(mu, ux0, ux1, uy0, uy1) <= __double2float_ru(r2)) atomicAdd(&counters[0], 1ull);
    }
    if (type == kWild) atomicAdd(&counters[1], 1ull);
    return;
  }
  if (type == kFallback) atomicAdd(&counters[2], 1ull);
  if (type == kWild) atomicAdd(&counters[3], 1ull);
  if (type == kDropped) atomicAdd(&counters[4], 1ull);

  // depth key and depth forms (rank order, Ind)
  // nominal depth: the depth row of A at the box centre applied to uw (the terms common
  // to all Gaussians, tau and beta, are left out: they cancel in depth differences)
  double cnom = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l) cnom += 0.5 * (pose.A[6 + l][0][kMaxP] + pose.A[6 + l][1][kMaxP]) * uw[l];
  const uint64_t key = order_key(dropped ? INFINITY : (prm.nominal_order ? cnom : dhi));
  key_out[oi] = key;
  key_sort[oi] = key;
  double *df = dform_out + oi * 2 * (kMaxP + 1);
  for (int k = 0; k <= kMaxP; ++k) { df[k] = 0.0; df[kMaxP + 1 + k] = 0.0; }
  for (int k = 0; k < P; ++k) { df[k] = d.lo[k]; df[kMaxP + 1 + k] = d.up[k]; }
  df[kMaxP] = d.lo[P];
  df[2 * kMaxP + 1] = d.up[P];
  dint_out[2 * oi] = cnom;
  dint_out[2 * oi + 1] = dhi;

  // record
  using R = Rec<P>;
  constexpr int F = R::F;
  double *rec = rec_out + oi * R::STRIDE;
  store_mr<P>(rec + R::DM, rec + R::DR, D2);
  store_mr<P>(rec + R::PM, rec + R::PR, DUP0);
  store_mr<P>(rec + R::PM + F, rec + R::PR + F, DUP1);
  double bmax[2] = {0.0, 0.0}, mb[2] = {0.0, 0.0};
  for (int e = 0; e < 6; ++e) {
    double *bm = rec + R::BM + F * e, *br = rec + R::BR + F * e, *cm = rec + R::CM + 4 * e;
    if (type == kNormal) {
      const int k = e / 3, nn = e % 3;
      const L64<P> b = l_add<P>(l_mul<P>(conic[k * 2 + 0], Mp0[nn]), l_mul<P>(conic[k * 2 + 1], Mp1[nn]));
      store_mr<P>(bm, br, b);
      double ylo, yhi;
      bounds_mr<P>(bm, br, ylo, yhi);
      // McCormick weights: c1 = (ylo + yhi)/2, c2 = (|yhi| - |ylo|)/2, c3 = (yhi - ylo)/2, c4 = (|ylo| + |yhi|)/2
      cm[0] = 0.5 * (ylo + yhi);
      cm[1] = 0.5 * (fabs(yhi) - fabs(ylo));
      cm[2] = 0.5 * (yhi - ylo);
      cm[3] = 0.5 * (fabs(ylo) + fabs(yhi));
      bmax[k] = fmax(bmax[k], fmax(fabs(ylo), fabs(yhi)));
      mb[k] = fmax(mb[k], mag_mr<P>(bm, br));
    } else {
      for (int j = 0; j < F; ++j) { bm[j] = 0.0; br[j] = 0.0; }
      for (int j = 0; j < 4; ++j) cm[j] = 0.0;
    }
  }
  const double slack = 1.0 + 0x1p-30;
  rec[R::MD2] = mag_mr<P>(rec + R::DM, rec + R::DR);
  for (int k = 0; k < 2; ++k) {
    rec[R::MDUP + k] = mag_mr<P>(rec + R::PM + F * k, rec + R::PR + F * k);
    rec[R::MBB + k] = slack * (mb[k] + 2.0 * bmax[k]);
    rec[R::BMAX + k] = slack * bmax[k];
  }
  rec[R::O] = (double)o;
  rec[R::OLO] = (double)sc.opac_lo[g];
  float *col = reinterpret_cast<float *>(rec + R::C);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    col[c] = sc.rgb[(size_t)c * n + g];
    col[3 + c] = sc.rgb_hi[(size_t)c * n + g];
  }
  const bool geo = (type == kNormal || type == kFallback);
  rec[R::LAM] = geo ? lam * (1.0 + 0x1p-40) : 0.0;
  float *pf = reinterpret_cast<float *>(rec + R::PRUNE);
  pf[0] = geo ? __double2float_rd(m0lo) : 0.0f;
  pf[1] = geo ? __double2float_ru(m0hi) : 0.0f;
  pf[2] = geo ? __double2float_rd(m1lo) : 0.0f;
  pf[3] = geo ? __double2float_ru(m1hi) : 0.0f;
  pf[4] = geo ? __double2float_ru(r2) : -1.0f;
  reinterpret_cast<int32_t *>(pf)[5] = type;
  for (int j = R::CM + 24; j < R::STRIDE; ++j) rec[j] = 0.0;

  // tile rectangle (inclusive) for binning; empty when the Gaussian cannot contribute
  int32_t *rc = rect_out + 4 * oi;
  if (type == kWild) {
    rc[0] = 0; rc[1] = 0; rc[2] = prm.ntx - 1; rc[3] = prm.nty - 1;
  } else if (!geo || r2 < 0.0) {
    rc[0] = 1; rc[1] = 1; rc[2] = 0; rc[3] = 0;
  } else {
    const double R = sqrt(r2) + 1.0;
    const double c0 = floor(m0lo - R + prm.cx - 0.5), c1 = ceil(m0hi + R + prm.cx - 0.5);
    const double r0 = floor(m1lo - R + prm.cy - 0.5), r1 = ceil(m1hi + R + prm.cy - 0.5);
    if (c1 < 0.0 || r1 < 0.0 || c0 > prm.width - 1 || r0 > prm.height - 1) {
      rc[0] = 1; rc[1] = 1; rc[2] = 0; rc[3] = 0;
    } else {
      const int ic0 = (int)fmax(c0, 0.0), ic1 = (int)fmin(c1, (double)(prm.width - 1));
      const int ir0 = (int)fmax(r0, 0.0), ir1 = (int)fmin(r1, (double)(prm.height - 1));
      rc[0] = ic0 / prm.tile; rc[1] = ir0 / prm.tile; rc[2] = ic1 / prm.tile; rc[3] = ir1 / prm.tile;
    }
  }
}

// one pose box: pose forms by value (kernel arguments)
template <int P>
__global__ __launch_bounds__(64) void k_project(SceneDev sc, const PoseForms pose, Params prm,
                                                double *__restrict__ rec_out, uint64_t *__restrict__ key_out,
                                                uint64_t *__restrict__ key_sort, uint32_t *__restrict__ perm_out,
                                                int32_t *__restrict__ rect_out, double *__restrict__ dform_out,
                                                double *__restrict__ dint_out, unsigned long long *__restrict__ counters) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= sc.n) return;
  project_one<P>(sc, pose, prm, g, (size_t)g, rec_out, key_out, key_sort, perm_out, rect_out, dform_out, dint_out,
                 counters, prm.eps_cull);
}

// several pose cells (grid.y): pose forms of cell c at poses[c] in device memory; with a
// table (cells of different scenes) cell c renders tab[c]'s scene at its items
template <int P>
__global__ __launch_bounds__(64) void k_project_cells(SceneDev sc, const PoseForms *__restrict__ poses, Params prm,
                                                      double *__restrict__ rec_out, uint64_t *__restrict__ key_out,
                                                      uint64_t *__restrict__ key_sort, uint32_t *__restrict__ perm_out,
                                                      int32_t *__restrict__ rect_out, double *__restrict__ dform_out,
                                                      double *__restrict__ dint_out,
                                                      unsigned long long *__restrict__ counters,
                                                      const CellScene *__restrict__ tab) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  const SceneDev &cs = cell_scene(sc, tab, c);
  if (g >= cs.n) return;
  project_one<P>(cs, poses[c], prm, g, cell_first(sc, tab, c) + g, rec_out, key_out, key_sort, perm_out, rect_out,
                 dform_out, dint_out, counters, tab ? tab[c].eps_cull : prm.eps_cull);
}

// Types only, for several pose cells (grid.y): counts[2c] = MatrixInv failures of cell c
// that the pruning test keeps somewhere in the image, counts[2c + 1] = its near-plane
// straddlers (the criteria of the adaptive refinement of a pose box).
template <int P>
__global__ __launch_bounds__(64) void k_classify_cells(SceneDev sc, const PoseForms *__restrict__ poses, Params prm,
                                                       unsigned long long *__restrict__ counts) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= sc.n) return;
  const int c = blockIdx.y;
  project_one<P, true>(sc, poses[c], prm, g, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                       counts + 2 * (size_t)c, prm.eps_cull);
}

// Pose forms on the host: O(1) work, passed to the kernels by value.
int pose_forms_host(const ar_pose_box &box, int P, PoseForms &out) {
  switch (P) {
    case 0: pose_forms<0>(box, out); return 0;
    case 1: pose_forms<1>(box, out); return 0;
    case 2: pose_forms<2>(box, out); return 0;
    case 3: pose_forms<3>(box, out); return 0;
    case 4: pose_forms<4>(box, out); return 0;
    case 5: pose_forms<5>(box, out); return 0;
    case 6: pose_forms<6>(box, out); return 0;
  }
  return -1;
}

template <int P>
static hipError_t launch_project_p(const SceneDev &sc, const PoseForms &pose, const PoseForms *poses_dev, int ncells,
                                   const Params &prm, Workspace &ws, hipStream_t s) {
  if (poses_dev) {
    int nmax = sc.n;   // the largest scene of the cells
    if (ws.tab)
      for (int c = 0; c < ncells; ++c) nmax = std::max(nmax, ws.tab_host[c].sc.n);
    hipLaunchKernelGGL(k_project_cells<P>, dim3((nmax + 63) / 64, ncells), dim3(64), 0, s, sc, poses_dev, prm, ws.rec,
                       ws.key, ws.key_sort, ws.perm, ws.rect, ws.dform, ws.dint, ws.counters, ws.tab);
  }
  else
    hipLaunchKernelGGL(k_project<P>, dim3((sc.n + 63) / 64), dim3(64), 0, s, sc, pose, prm, ws.rec, ws.key,
                       ws.key_sort, ws.perm, ws.rect, ws.dform, ws.dint, ws.counters);
  return hipGetLastError();
}

hipError_t launch_project(int P, const SceneDev &sc, const PoseForms &pose, const PoseForms *poses_dev, int ncells,
                          const Params &prm, Workspace &ws,
                          hipStream_t s) {
  switch (P) {
    case 0: return launch_project_p<0>(sc, pose, poses_dev, ncells, prm, ws, s);
    case 1: return launch_project_p<1>(sc, pose, poses_dev, ncells, prm, ws, s);
    case 2: return launch_project_p<2>(sc, pose, poses_dev, ncells, prm, ws, s);
    case 3: return launch_project_p<3>(sc, pose, poses_dev, ncells, prm, ws, s);
    case 4: return launch_project_p<4>(sc, pose, poses_dev, ncells, prm, ws, s);
    case 5: return launch_project_p<5>(sc, pose, poses_dev, ncells, prm, ws, s);
    case 6: return launch_project_p<6>(sc, pose, poses_dev, ncells, prm, ws, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_classify(int P, const SceneDev &sc, const PoseForms *poses_dev, int ncells, const Params &prm,
                           unsigned long long *counts, hipStream_t s) {
  const dim3 grid((unsigned)((sc.n + 63) / 64), (unsigned)ncells);
  switch (P) {
    case 0: hipLaunchKernelGGL(k_classify_cells<0>, grid, dim3(64), 0, s, sc, poses_dev, prm, counts); break;
    case 1: hipLaunchKernelGGL(k_classify_cells<1>, grid, dim3(64), 0, s, sc, poses_dev, prm, counts); break;
    case 2: hipLaunchKernelGGL(k_classify_cells<2>, grid, dim3(64), 0, s, sc, poses_dev, prm, counts); break;
    case 3: hipLaunchKernelGGL(k_classify_cells<3>, grid, dim3(64), 0, s, sc, poses_dev, prm, counts); break;
    case 4: hipLaunchKernelGGL(k_classify_cells<4>, grid, dim3(64), 0, s, sc, poses_dev, prm, counts); break;
    case 5: hipLaunchKernelGGL(k_classify_cells<5>, grid, dim3(64), 0, s, sc, poses_dev, prm, counts); break;
    case 6: hipLaunchKernelGGL(k_classify_cells<6>, grid, dim3(64), 0, s, sc, poses_dev, prm, counts); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ar
