// Tree-level |M|^2 of the quark-initiated top-pair + jet channels (HIP,
// gfx950): q(p1) q~(p2) -> t t~ g(k) and q(p1) g(p2) -> t t~ q(k).
//
// Two fermion lines (the light quark line and the top line) joined by one
// gluon, with one more external gluon attached to either line or to the
// connecting gluon through the three-gluon vertex: five Feynman diagrams
// (Feynman gauge).  Their Lorentz parts K_d are built per helicity state from
// the chiral-basis spinors and vertex/propagator forms of amp.h and the
// vector currents psibar gamma^mu chi; their colour factors enter through the
// exact matrix CC[d][d'] = sum_colours C_d C_d'^* (gen/colour_qq.h), so that
// sum_colours |M|^2 = sum_{d,d'} K_d K_d'^* CC[d][d'] (the helicity loop and
// the colour aggregation of Sec. 2.2).  Row spinors times real vectors use
// psibar Jslash = dbar(Jslash psi), valid for real J.  Coupling g = 1.
#pragma once
#include "amp.h"
#include "gen/colour_qq.h"

namespace mf {

// Complex four-vector (contravariant components).
template <class R> struct CV4 {
  C2<R> c[4];
};
template <class R> __device__ __forceinline__ CV4<R> vcur(const Sp<R>& row, const Sp<R>& col) {
  // row gamma^mu col, gamma^mu = [[0, sigma^mu], [sigmabar^mu, 0]]
  CV4<R> j;
  j.c[0] = cmul(row.s0, col.s2) + cmul(row.s1, col.s3) + cmul(row.s2, col.s0) + cmul(row.s3, col.s1);
  j.c[1] = (cmul(row.s0, col.s3) + cmul(row.s1, col.s2)) - (cmul(row.s2, col.s1) + cmul(row.s3, col.s0));
  const C2<R> a = cmul(row.s1, col.s2) - cmul(row.s0, col.s3);
  const C2<R> b = cmul(row.s2, col.s1) - cmul(row.s3, col.s0);
  const C2<R> ab = a + b;
  j.c[2] = C2<R>{R(0.0) - ab.im, ab.re};
  j.c[3] = (cmul(row.s0, col.s2) - cmul(row.s1, col.s3)) - (cmul(row.s2, col.s0) - cmul(row.s3, col.s1));
  return j;
}
template <class R> __device__ __forceinline__ C2<R> mdotc(const CV4<R>& a, const CV4<R>& b) {
  return cmul(a.c[0], b.c[0]) - cmul(a.c[1], b.c[1]) - cmul(a.c[2], b.c[2]) - cmul(a.c[3], b.c[3]);
}
template <class R> __device__ __forceinline__ C2<R> mdotr(const V4<R>& a, const CV4<R>& b) {
  return C2<R>{a.t * b.c[0].re - a.x * b.c[1].re - a.y * b.c[2].re - a.z * b.c[3].re,
               a.t * b.c[0].im - a.x * b.c[1].im - a.y * b.c[2].im - a.z * b.c[3].im};
}
template <class R> __device__ __forceinline__ Sp<R> sbar(const Sp<R>& p) {
  // psi^dagger gamma^0 in the chiral basis
  return Sp<R>{C2<R>{p.s2.re, R(0.0) - p.s2.im}, C2<R>{p.s3.re, R(0.0) - p.s3.im},
               C2<R>{p.s0.re, R(0.0) - p.s0.im}, C2<R>{p.s1.re, R(0.0) - p.s1.im}};
}
template <class R> __device__ __forceinline__ C2<R> cscale(C2<R> a, R s) { return C2<R>{a.re * s, a.im * s}; }
// -i z
template <class R> __device__ __forceinline__ C2<R> mul_mi(C2<R> z) { return C2<R>{z.im, R(0.0) - z.re}; }

// Three-gluon vertex contracted with its legs (a: real polarisation e with
// incoming momentum k; b, c: currents X, Y with incoming momenta p, q):
//   (e.X)((k - p).Y) + (X.Y)((p - q).e) + (Y.e)((q - k).X)
template <class R>
__device__ __forceinline__ C2<R> vertex3(const V4<R>& e, const V4<R>& k, const CV4<R>& X, const V4<R>& p,
                                         const CV4<R>& Y, const V4<R>& q) {
  const C2<R> eX = mdotr(e, X), eY = mdotr(e, Y), XY = mdotc(X, Y);
  const C2<R> kpY = mdotr(k - p, Y), qkX = mdotr(q - k, X);
  const R pqe = mdot(p - q, e);
  return cmul(eX, kpY) + cscale(XY, pqe) + cmul(eY, qkX);
}

// sum_{d,d'} Re(K_d K_d'^* CC[d][d']) with the exact Hermitian matrix
// CC = (QQ_CC_RE + i QQ_CC_IM) / QQ_CC_DEN.
template <class R> __device__ __forceinline__ R colour_form5(const C2<R>* K) {
  R t = R(0.0);
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    t = t + R(QQ_CC_RE[d * 5 + d]) * cabs2(K[d]);
#pragma unroll
    for (int e = d + 1; e < 5; ++e) {
      // 2 Re(K_d K_e^* CC[d][e])
      const C2<R> z = C2<R>{K[d].re * K[e].re + K[d].im * K[e].im, K[d].im * K[e].re - K[d].re * K[e].im};
      t = t + R(2.0) * (R(QQ_CC_RE[d * 5 + e]) * z.re - R(QQ_CC_IM[d * 5 + e]) * z.im);
    }
  }
  return t * R(1.0 / QQ_CC_DEN);
}

// q(p1) q~(p2) -> t(pt) t~(ptb) g(k): colour- and helicity-summed |M|^2, g = 1.
template <class R>
__device__ __forceinline__ R me_qqbar_g(const V4<R>& p1, const V4<R>& p2, const V4<R>& pt, const V4<R>& ptb,
                                        const V4<R>& k, R mt) {
  const R z = R(0.0);
  const V4<R> q12 = p1 + p2, q34 = pt + ptb;
  const R s12 = mdot(q12, q12), s34 = mdot(q34, q34);
  const V4<R> a1 = p1 - k, a2 = k - p2, a3 = pt + k, a4 = z * k - (ptb + k);
  const R i1 = R(1.0) / (mdot(a1, a1) * s34), i2 = R(1.0) / (mdot(a2, a2) * s34);
  const R f3 = R(1.0) / (mdot(a3, a3) - mt * mt), f4 = R(1.0) / (mdot(a4, a4) - mt * mt);
  const R i12 = R(1.0) / s12, i5 = R(1.0) / (s12 * s34);
  const V4<R> mk = z * k - k, mq34 = z * q34 - q34;
  V4<R> E[2];
  lin_pols(k, E);
  R total = R(0.0);
#pragma unroll 1
  for (int h = 0; h < 16; ++h) {
    const int l1 = (h & 8) ? 1 : -1, l2 = (h & 4) ? 1 : -1, l3 = (h & 2) ? 1 : -1, l4 = (h & 1) ? 1 : -1;
    const Sp<R> u1 = sbar(ubar_spinor(p1, z, l1));
    const Sp<R> v2 = v_spinor(p2, z, l2);
    const Sp<R> vb2 = sbar(v2);
    const Sp<R> ub3 = ubar_spinor(pt, mt, l3);
    const Sp<R> u3 = sbar(ub3);
    const Sp<R> v4 = v_spinor(ptb, mt, l4);
    const CV4<R> J12 = vcur(vb2, u1), J34 = vcur(ub3, v4);
#pragma unroll 1
    for (int pol = 0; pol < 2; ++pol) {
      const V4<R> e = pol ? E[1] : E[0];
      C2<R> K[5];
      // emission from the incoming quark, then from the incoming antiquark
      K[0] = mul_mi(cscale(mdotc(vcur(vb2, slash(a1, slash(e, u1))), J34), i1));
      K[1] = mul_mi(cscale(mdotc(vcur(sbar(slash(a2, slash(e, v2))), u1), J34), i2));
      // emission from the top, then from the antitop
      K[2] = mul_mi(cscale(mdotc(vcur(sbar(prop(a3, mt, f3, slash(e, u3))), v4), J12), i12));
      K[3] = mul_mi(cscale(mdotc(vcur(ub3, prop(a4, mt, f4, slash(e, v4))), J12), i12));
      // three-gluon vertex: (e, -k), (J12, p1 + p2), (J34, -(pt + ptb))
      K[4] = cscale(vertex3(e, mk, J12, q12, J34, mq34), i5);
      total = total + colour_form5(K);
    }
  }
  return total;
}

// q(p1) g(p2) -> t(pt) t~(ptb) q(k): colour- and helicity-summed |M|^2, g = 1.
template <class R>
__device__ __forceinline__ R me_qg_q(const V4<R>& p1, const V4<R>& p2, const V4<R>& pt, const V4<R>& ptb,
                                     const V4<R>& k, R mt) {
  const R z = R(0.0);
  const V4<R> q12 = p1 + p2, q34 = pt + ptb, q15 = p1 - k;
  const R s12 = mdot(q12, q12), s34 = mdot(q34, q34), t15 = mdot(q15, q15);
  const V4<R> a2 = k - p2, a3 = pt - p2, a4 = p2 - ptb;
  const R i0 = R(1.0) / (s12 * s34), i2 = R(1.0) / (mdot(a2, a2) * s34);
  const R f3 = R(1.0) / (mdot(a3, a3) - mt * mt), f4 = R(1.0) / (mdot(a4, a4) - mt * mt);
  const R i15 = R(1.0) / t15, i5 = R(1.0) / (t15 * s34);
  const V4<R> mq34 = z * q34 - q34;
  V4<R> E[2];
  lin_pols(p2, E);
  R total = R(0.0);
#pragma unroll 1
  for (int h = 0; h < 16; ++h) {
    const int l1 = (h & 8) ? 1 : -1, l5 = (h & 4) ? 1 : -1, l3 = (h & 2) ? 1 : -1, l4 = (h & 1) ? 1 : -1;
    const Sp<R> u1 = sbar(ubar_spinor(p1, z, l1));
    const Sp<R> ub5 = ubar_spinor(k, z, l5);
    const Sp<R> u5 = sbar(ub5);
    const Sp<R> ub3 = ubar_spinor(pt, mt, l3);
    const Sp<R> u3 = sbar(ub3);
    const Sp<R> v4 = v_spinor(ptb, mt, l4);
    const CV4<R> J15 = vcur(ub5, u1), J34 = vcur(ub3, v4);
#pragma unroll 1
    for (int pol = 0; pol < 2; ++pol) {
      const V4<R> e = pol ? E[1] : E[0];
      C2<R> K[5];
      // the gluon absorbed by the quark line before / after the top pair leaves it
      K[0] = mul_mi(cscale(mdotc(vcur(ub5, slash(q12, slash(e, u1))), J34), i0));
      K[1] = mul_mi(cscale(mdotc(vcur(sbar(slash(a2, slash(e, u5))), u1), J34), i2));
      // the gluon absorbed by the top line next to the top / the antitop
      K[2] = mul_mi(cscale(mdotc(vcur(sbar(prop(a3, mt, f3, slash(e, u3))), v4), J15), i15));
      K[3] = mul_mi(cscale(mdotc(vcur(ub3, prop(a4, mt, f4, slash(e, v4))), J15), i15));
      // three-gluon vertex: (e, p2), (J15, p1 - k), (J34, -(pt + ptb))
      K[4] = cscale(vertex3(e, p2, J15, q15, J34, mq34), i5);
      total = total + colour_form5(K);
    }
  }
  return total;
}

}  // namespace mf
