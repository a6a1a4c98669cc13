// BlendInd colour accumulation shared by the pixel loops (device code).
//
// The pc step of Alg. BlendInd, pc = sum_i T_i a_i c_i, with interval transmittances
// [T_lo, T_hi] and linear-form alphas: the lower image accumulates the forms
// c_i T_lo[i] a_i^lower(e), the upper image c_i T_hi[i] a_i^upper(e) and the interval
// sum c_i T_hi[i] a_hi[i].  Sums are FP64; magnitude sums in FP32 bound their rounding.
#pragma once

#include "ar_pair.h"

namespace ar {

// Partial result of one segment, NF columns of 64 doubles (one per pixel lane).
template <int P>
struct Part {
  static constexpr int F = P + 1;
  static constexpr int LO = 0;               // [3][F] lower colour forms
  static constexpr int HI = 3 * F;           // [3][F] upper colour forms
  static constexpr int IHI = 6 * F;          // [3] interval upper sums
  static constexpr int TLO = 6 * F + 3;      // segment transmittance products
  static constexpr int THI = 6 * F + 4;
  static constexpr int MAG = 6 * F + 5;      // magnitude sums (two floats)
  static constexpr int STOP = 6 * F + 6;     // 1 when the segment stopped early
  static constexpr int CNT = 6 * F + 7;      // evaluated pairs of the wave (same in every lane)
  static constexpr int NF = 6 * F + 8;
};

template <int P>
struct Acc {
  double lo[3][P + 1];
  double hi[3][P + 1];
  double ihi[3];
  float magl, magh;  // magnitude sums bounding the FP64 rounding of the sums
};

template <int P>
__device__ __forceinline__ void acc_zero(Acc<P> &a) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int j = 0; j <= P; ++j) { a.lo[c][j] = 0.0; a.hi[c][j] = 0.0; }
    a.ihi[c] = 0.0;
  }
  a.magl = 0.0f;
  a.magh = 0.0f;
}

// Alpha interval of a MatrixInv fallback (footprint bound) or a near-plane straddler.
template <int P>
__device__ __forceinline__ double alpha_hi_special(const double *__restrict__ rec, int type, double ux, double uy,
                                                   const double *cf) {
  using R = Rec<P>;
  const double o = rec[R::O];
  if (type != kFallback) return o;
  const double d2 = dist2_box64(rec_prune<P>(rec), ux, uy);
  const double lam = rec[R::LAM];
  double e_dn, e_up;
  exp_encl(-0.5 * d2 * (1.0 - 8.0 * kU) / lam, e_dn, e_up, cf);
  return fmin(o, o * e_up * (1.0 + 4.0 * kU));
}

// Alpha of one (pixel, Gaussian) pair as linear forms: lower form gl, upper form gh,
// interval [a_lo, a_hi] and the magnitudes ml >= |gl|, mh >= |gh| + a_hi (for the
// rounding bound of the sums).  Zero when the pair is not kept.
template <int P>
struct PairAlpha {
  double gl[P + 1], gh[P + 1];
  double a_lo, a_hi;
  float ml, mh;
};

template <int P>
__device__ __forceinline__ void pair_alpha(const double *__restrict__ rec, int type, bool kept, double ux, double uy,
                                           PairAlpha<P> &pa, const double *cf) {
  using R = Rec<P>;
#pragma unroll
  for (int j = 0; j <= P; ++j) { pa.gl[j] = 0.0; pa.gh[j] = 0.0; }
  pa.a_lo = 0.0;
  pa.a_hi = 0.0;
  pa.ml = 0.0f;
  pa.mh = 0.0f;
  const double o = rec[R::O];
  if (type == kNormal) {
    if (kept) {
      SForms<P> s;
      s_forms<P>(rec, ux, uy, s);
      ExpBounds b;
      exp_bounds(s.slo, s.shi, rec[R::OLO], o, b, cf);
      // lower alpha form  o_lo e_dn (x_lower(e) - xlo + 1),  x_lower = -s_upper / 2
      // upper alpha form  o e_up + o k_up (x_upper(e) - xlo),  x_upper = -s_lower / 2
      // (o_lo, o: the opacity interval; equal for a plain scene)
      const double wl = rec[R::OLO] * b.e_dn;
      const double wk = o * b.k_up;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        pa.gl[j] = wl * (-0.5 * s.sh[j]);
        pa.gh[j] = wk * (-0.5 * s.sl[j]);
      }
      pa.gl[P] = wl * ((-0.5 * s.sh[P] - b.xlo) + 1.0);
      pa.gh[P] = o * b.e_up + wk * (-0.5 * s.sl[P] - b.xlo);
      pa.ml = (float)(wl * (0.5 * s.msh + fabs(b.xlo) + 1.0));
      pa.mh = (float)(o * b.e_up + wk * (0.5 * s.msl + fabs(b.xlo)) + b.a_hi);
      pa.a_lo = b.a_lo;
      pa.a_hi = b.a_hi;
    }
  } else if (kept) {
    // MatrixInv fallback: [0, footprint bound]; near-plane straddler: [0, o]
    const double ah = alpha_hi_special<P>(rec, type, ux, uy, cf);
    pa.gh[P] = ah;
    pa.a_hi = ah;
    pa.mh = 2.0f * (float)ah;
  }
}

// BlendInd contribution of one pair with the transmittances (tlo, thi) in front:
// colour forms c_lo T_lo gl, c_hi T_hi gh and the interval sum c_hi T_hi a_hi (c_lo = c_hi
// = c for a plain scene).
template <int P>
__device__ __forceinline__ void acc_pair(Acc<P> &acc, const double *__restrict__ rec, const PairAlpha<P> &pa,
                                         double tlo, double thi) {
  using R = Rec<P>;
  const float *col = reinterpret_cast<const float *>(rec + R::C);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double wlo = (double)col[c] * tlo, whi = (double)col[3 + c] * thi;
#pragma unroll
    for (int j = 0; j <= P; ++j) {
      acc.lo[c][j] = fma(wlo, pa.gl[j], acc.lo[c][j]);
      acc.hi[c][j] = fma(whi, pa.gh[j], acc.hi[c][j]);
    }
    acc.ihi[c] = fma(whi, pa.a_hi, acc.ihi[c]);
  }
  acc.magl = fmaf((float)tlo, pa.ml, acc.magl) * (1.0f + 4.0f * kU32);
  acc.magh = fmaf((float)thi, pa.mh, acc.magh) * (1.0f + 4.0f * kU32);
}

// One (pixel, Gaussian) pair: alpha bounds and its BlendInd contribution with the
// transmittances (tlo, thi) of the Gaussians in front.  Returns the alpha interval.
template <int P>
__device__ __forceinline__ void pair_contrib(const double *__restrict__ rec, int type, double ux, double uy,
                                             double tlo, double thi, Acc<P> &acc, double &a_lo, double &a_hi,
                                             const double *cf) {
  PairAlpha<P> pa;
  pair_alpha<P>(rec, type, true, ux, uy, pa, cf);
  acc_pair<P>(acc, rec, pa, tlo, thi);
  a_lo = pa.a_lo;
  a_hi = pa.a_hi;
}

// Alpha interval of one pair without the colour forms (types as in pair_contrib).
template <int P>
__device__ __forceinline__ void alpha_interval(const double *__restrict__ rec, int type, double ux, double uy,
                                               double &a_lo, double &a_hi, const double *cf) {
  using R = Rec<P>;
  if (type == kNormal) {
    SForms<P> s;
    s_forms<P>(rec, ux, uy, s);
    ExpBounds b;
    exp_bounds(s.slo, s.shi, rec[R::OLO], rec[R::O], b, cf);
    a_lo = b.a_lo;
    a_hi = b.a_hi;
  } else {
    a_lo = 0.0;
    a_hi = alpha_hi_special<P>(rec, type, ux, uy, cf);
  }
}

// Item and pruning data (box, r2, type) of up to 64 upcoming list positions, one lane
// each, and optionally their depth keys, fetched with vector loads; the pixel loops
// read them back with readlane, so no dependent scalar load stands between two pairs.
struct Lookahead {
  uint32_t gv = 0, klo = ~0u, khi = ~0u;
  int4 bv = make_int4(0, 0, 0, 0);
  int rv = 0, tv = 0;

  template <int P>
  __device__ __forceinline__ void fetch(const double *__restrict__ recs, const uint32_t *__restrict__ items, int pos,
                                        int end, const uint64_t *__restrict__ keys = nullptr) {
    if (pos < end) {
      gv = items[pos];
      if (keys) {
        const uint64_t kk = keys[gv];
        klo = (uint32_t)kk;
        khi = (uint32_t)(kk >> 32);
      }
      const int32_t *ph = reinterpret_cast<const int32_t *>(recs + (size_t)gv * Rec<P>::STRIDE + Rec<P>::PRUNE);
      bv = *reinterpret_cast<const int4 *>(ph);
      const int2 rt = *reinterpret_cast<const int2 *>(ph + 4);
      rv = rt.x;
      tv = rt.y;
    }
  }
  __device__ __forceinline__ uint32_t gid(int k) const { return (uint32_t)__builtin_amdgcn_readlane((int)gv, k); }
  __device__ __forceinline__ uint64_t key(int k) const {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)khi, k) << 32) |
           (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)klo, k);
  }
  __device__ __forceinline__ int type(int k) const { return __builtin_amdgcn_readlane(tv, k); }
  // the pruning test of the pair (float32, as in the binning)
  __device__ __forceinline__ bool kept(int k, int type, float ux, float uy) const {
    if (type == kWild) return true;
    const float b0 = __int_as_float(__builtin_amdgcn_readlane(bv.x, k));
    const float b1 = __int_as_float(__builtin_amdgcn_readlane(bv.y, k));
    const float b2 = __int_as_float(__builtin_amdgcn_readlane(bv.z, k));
    const float b3 = __int_as_float(__builtin_amdgcn_readlane(bv.w, k));
    const float r2 = __int_as_float(__builtin_amdgcn_readlane(rv, k));
    return dist2_box(b0, b1, b2, b3, ux, uy) <= r2;
  }
};

// Concretise one colour channel's forms over the box and write the pixel's lower / upper
// value.  nterm bounds the number of summed terms (for the FP64 rounding bound); extra_hi
// is added to the upper bound (the transmittance left when a segment stops early).
template <int P>
__device__ __forceinline__ void write_channel(const double *lo_f, const double *hi_f, double ihi, float magl, float magh,
                                              double nterm, double E, double extra_hi, float *out_lo, float *out_hi,
                                              size_t idx) {
  const double wlo = (nterm + 16.0) * 0x1p-51 * (double)magl;
  const double whi = (nterm + 16.0) * 0x1p-51 * (double)magh;
  double sl = 0.0, sh = 0.0;
#pragma unroll
  for (int j = 0; j < P; ++j) { sl += fabs(lo_f[j]); sh += fabs(hi_f[j]); }
  double lo = lo_f[P] - sl - E - wlo;
  double hi = fmin(hi_f[P] + sh, ihi) + E + whi + extra_hi;
  lo = fmin(fmax(lo, 0.0), 1.0);
  hi = fmin(fmax(hi, 0.0), 1.0);
  out_lo[idx] = __double2float_rd(lo);
  out_hi[idx] = __double2float_ru(hi);
}

}  // namespace ar
