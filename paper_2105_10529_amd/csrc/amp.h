// Device arithmetic for helicity amplitudes on gfx950 (HIP).
//
// Real four-vectors, complex numbers, Dirac spinors in the chiral
// representation, the colour-ordered vertex routines used by the generated
// amplitude code, external wavefunctions (Sec. 2.2: wavefunctions and
// vertices, written branch-free so that a wavefront of events never
// diverges), and a forward-mode dual number for derivatives.
//
// Conventions: metric (+,-,-,-); all momenta outgoing inside the amplitude;
// gamma^0 = [[0,1],[1,0]], gamma^k = [[0,s^k],[-s^k,0]].
#pragma once
#include <hip/hip_runtime.h>

namespace mf {

// ------------------------------------------------------------ dual numbers
// One tangent direction; used with R = double or float.
template <class T> struct Dual {
  T v, d;
  __host__ __device__ Dual() : v(T(0)), d(T(0)) {}
  __host__ __device__ Dual(T a) : v(a), d(T(0)) {}
  __host__ __device__ Dual(T a, T b) : v(a), d(b) {}
};
template <class T> __device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return Dual<T>(a.v + b.v, a.d + b.d); }
template <class T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return Dual<T>(a.v - b.v, a.d - b.d); }
template <class T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return Dual<T>(-a.v, -a.d); }
template <class T> __device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) {
  return Dual<T>(a.v * b.v, fma(a.d, b.v, a.v * b.d));
}
template <class T> __device__ __forceinline__ Dual<T> operator/(Dual<T> a, Dual<T> b) {
  T iv = T(1) / b.v;
  T q = a.v * iv;
  return Dual<T>(q, (a.d - q * b.d) * iv);
}
__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ float val(float x) { return x; }
template <class T> __device__ __forceinline__ T val(Dual<T> x) { return x.v; }
__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float dsqrt(float x) { return sqrtf(x); }
template <class T> __device__ __forceinline__ Dual<T> dsqrt(Dual<T> x) {
  T s = dsqrt(x.v);
  return Dual<T>(s, s > T(0) ? x.d / (T(2) * s) : T(0));
}
__device__ __forceinline__ double dlog(double x) { return log(x); }
template <class T> __device__ __forceinline__ Dual<T> dlog(Dual<T> x) { return Dual<T>(dlog(x.v), x.d / x.v); }

// Conversion from the kinematic type (FP64 or its dual) to the amplitude type.
template <class R> __device__ __forceinline__ R cvt(double x) { return R(x); }
template <> __device__ __forceinline__ float cvt<float>(double x) { return (float)x; }
template <class R> __device__ __forceinline__ R cvt(Dual<double> x);
template <> __device__ __forceinline__ Dual<double> cvt<Dual<double>>(Dual<double> x) { return x; }
template <> __device__ __forceinline__ Dual<float> cvt<Dual<float>>(Dual<double> x) {
  return Dual<float>((float)x.v, (float)x.d);
}

// ------------------------------------------------------------ four-vectors
template <class R> struct V4 {
  R t, x, y, z;
};
template <class R> __device__ __forceinline__ V4<R> operator+(const V4<R>& a, const V4<R>& b) {
  return V4<R>{a.t + b.t, a.x + b.x, a.y + b.y, a.z + b.z};
}
template <class R> __device__ __forceinline__ V4<R> operator-(const V4<R>& a, const V4<R>& b) {
  return V4<R>{a.t - b.t, a.x - b.x, a.y - b.y, a.z - b.z};
}
template <class R> __device__ __forceinline__ V4<R> operator*(R s, const V4<R>& a) {
  return V4<R>{s * a.t, s * a.x, s * a.y, s * a.z};
}
template <class R> __device__ __forceinline__ R mdot(const V4<R>& a, const V4<R>& b) {
  return a.t * b.t - a.x * b.x - a.y * b.y - a.z * b.z;
}

template <class R, class RK> __device__ __forceinline__ V4<R> cvt4(const V4<RK>& p) {
  return V4<R>{cvt<R>(p.t), cvt<R>(p.x), cvt<R>(p.y), cvt<R>(p.z)};
}

// Opaque copies: the compiler must treat the value as redefined here, so
// expressions built from it are neither merged with earlier ones nor hoisted
// out of the enclosing loop.  Used by the generated amplitude code to bound
// register lifetimes.
__device__ __forceinline__ void opaque(float& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void opaque(double& x) { asm volatile("" : "+v"(x)); }
template <class T> __device__ __forceinline__ void opaque(Dual<T>& x) {
  opaque(x.v);
  opaque(x.d);
}
template <class R> __device__ __forceinline__ void opaque4(V4<R>& p) {
  opaque(p.t);
  opaque(p.x);
  opaque(p.y);
  opaque(p.z);
}

// Colour-ordered three-gluon vertex contracted with two currents X, Y of
// outgoing momenta PX, PY (coupling and the off-shell propagator excluded):
//   X (2PX+PY).Y + (X.Y)(PY-PX) - Y (PX+2PY).X
// X and Y are always complete Berends-Giele currents (or polarisation
// vectors) of on-shell transverse gluons, which are conserved, PX.X =
// PY.Y = 0, so the coefficients are formed as 2 PX.Y and 2 PY.X.
template <class R>
__device__ __forceinline__ V4<R> v3(const V4<R>& X, const V4<R>& Y, const V4<R>& PX, const V4<R>& PY) {
  R a = R(2.0) * mdot(PX, Y);
  R d = R(2.0) * mdot(PY, X);
  R c = mdot(X, Y);
  return V4<R>{a * X.t + c * (PY.t - PX.t) - d * Y.t, a * X.x + c * (PY.x - PX.x) - d * Y.x,
               a * X.y + c * (PY.y - PX.y) - d * Y.y, a * X.z + c * (PY.z - PX.z) - d * Y.z};
}
// o + v3(X, Y, PX, PY): the vertex added into an accumulated current, each
// component one chain of fused multiply-adds (sums of vertices are formed
// this way instead of adding separately rounded vertices).
template <class R>
__device__ __forceinline__ V4<R> v3_acc(const V4<R>& X, const V4<R>& Y, const V4<R>& PX, const V4<R>& PY, V4<R> o) {
  R a = R(2.0) * mdot(PX, Y);
  R d = R(2.0) * mdot(PY, X);
  R c = mdot(X, Y);
  o.t = ((o.t + a * X.t) + c * (PY.t - PX.t)) - d * Y.t;
  o.x = ((o.x + a * X.x) + c * (PY.x - PX.x)) - d * Y.x;
  o.y = ((o.y + a * X.y) + c * (PY.y - PX.y)) - d * Y.y;
  o.z = ((o.z + a * X.z) + c * (PY.z - PX.z)) - d * Y.z;
  return o;
}
// Colour-ordered four-gluon vertex with three adjacent currents:
//   2B(A.C) - A(B.C) - C(A.B)
template <class R> __device__ __forceinline__ V4<R> w4(const V4<R>& A, const V4<R>& B, const V4<R>& C) {
  R ac = R(2.0) * mdot(A, C), bc = mdot(B, C), ab = mdot(A, B);
  return V4<R>{ac * B.t - bc * A.t - ab * C.t, ac * B.x - bc * A.x - ab * C.x, ac * B.y - bc * A.y - ab * C.y,
               ac * B.z - bc * A.z - ab * C.z};
}

// o - w4(A, B, C) as chains of fused multiply-adds.
template <class R>
__device__ __forceinline__ V4<R> w4_sub(const V4<R>& A, const V4<R>& B, const V4<R>& C, V4<R> o) {
  R ac = R(2.0) * mdot(A, C), bc = mdot(B, C), ab = mdot(A, B);
  o.t = ((o.t - ac * B.t) + bc * A.t) + ab * C.t;
  o.x = ((o.x - ac * B.x) + bc * A.x) + ab * C.x;
  o.y = ((o.y - ac * B.y) + bc * A.y) + ab * C.y;
  o.z = ((o.z - ac * B.z) + bc * A.z) + ab * C.z;
  return o;
}

// ---------------------------------------------------------------- complex
template <class R> struct C2 {
  R re, im;
};
template <class R> __device__ __forceinline__ C2<R> operator+(C2<R> a, C2<R> b) { return C2<R>{a.re + b.re, a.im + b.im}; }
template <class R> __device__ __forceinline__ C2<R> operator-(C2<R> a, C2<R> b) { return C2<R>{a.re - b.re, a.im - b.im}; }
template <class R> __device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
  return C2<R>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> __device__ __forceinline__ R cabs2(C2<R> a) { return a.re * a.re + a.im * a.im; }
// Re(a^* b)
template <class R> __device__ __forceinline__ R cre_dot(C2<R> a, C2<R> b) { return a.re * b.re + a.im * b.im; }
// acc + |a|^2 and acc + Re(a^* b), two fused multiply-adds each
template <class R> __device__ __forceinline__ R cabs2_acc(C2<R> a, R acc) { return (acc + a.re * a.re) + a.im * a.im; }
template <class R> __device__ __forceinline__ R cre_dot_acc(C2<R> a, C2<R> b, R acc) {
  return (acc + a.re * b.re) + a.im * b.im;
}

// ---------------------------------------------------------------- spinors
template <class R> struct Sp {
  C2<R> s0, s1, s2, s3;
};
template <class R> __device__ __forceinline__ Sp<R> operator+(const Sp<R>& a, const Sp<R>& b) {
  return Sp<R>{a.s0 + b.s0, a.s1 + b.s1, a.s2 + b.s2, a.s3 + b.s3};
}
// slash(J) psi for a real four-vector J.
//   out0 = (J0-J3) p2 - (J1 - i J2) p3     out2 = (J0+J3) p0 + (J1 - i J2) p1
//   out1 = -(J1 + i J2) p2 + (J0+J3) p3    out3 = (J1 + i J2) p0 + (J0-J3) p1
template <class R> __device__ __forceinline__ Sp<R> slash(const V4<R>& J, const Sp<R>& p) {
  R a = J.t - J.z, b = J.t + J.z, c = J.x, d = J.y;
  Sp<R> o;
  // (c - i d)(x + i y) = (c x + d y) + i (c y - d x);  (c + i d)(x + i y) = (c x - d y) + i (c y + d x)
  o.s0 = C2<R>{a * p.s2.re - (c * p.s3.re + d * p.s3.im), a * p.s2.im - (c * p.s3.im - d * p.s3.re)};
  o.s1 = C2<R>{b * p.s3.re - (c * p.s2.re - d * p.s2.im), b * p.s3.im - (c * p.s2.im + d * p.s2.re)};
  o.s2 = C2<R>{b * p.s0.re + (c * p.s1.re + d * p.s1.im), b * p.s0.im + (c * p.s1.im - d * p.s1.re)};
  o.s3 = C2<R>{a * p.s1.re + (c * p.s0.re - d * p.s0.im), a * p.s1.im + (c * p.s0.im + d * p.s0.re)};
  return o;
}
// o + slash(J) psi, each component one chain of fused multiply-adds.
template <class R> __device__ __forceinline__ Sp<R> slash_acc(const V4<R>& J, const Sp<R>& p, Sp<R> o) {
  R a = J.t - J.z, b = J.t + J.z, c = J.x, d = J.y;
  o.s0.re = ((o.s0.re + a * p.s2.re) - c * p.s3.re) - d * p.s3.im;
  o.s0.im = ((o.s0.im + a * p.s2.im) - c * p.s3.im) + d * p.s3.re;
  o.s1.re = ((o.s1.re + b * p.s3.re) - c * p.s2.re) + d * p.s2.im;
  o.s1.im = ((o.s1.im + b * p.s3.im) - c * p.s2.im) - d * p.s2.re;
  o.s2.re = ((o.s2.re + b * p.s0.re) + c * p.s1.re) + d * p.s1.im;
  o.s2.im = ((o.s2.im + b * p.s0.im) + c * p.s1.im) - d * p.s1.re;
  o.s3.re = ((o.s3.re + a * p.s1.re) + c * p.s0.re) - d * p.s0.im;
  o.s3.im = ((o.s3.im + a * p.s1.im) + c * p.s0.im) + d * p.s0.re;
  return o;
}
// fm phi + slash(J) phi with the slash given by its coefficients
// a = J0 - J3, b = J0 + J3, c = J1, d = J2 (already scaled by the caller).
template <class R> __device__ __forceinline__ Sp<R> pslash(R fm, R a, R b, R c, R d, const Sp<R>& p) {
  Sp<R> o;
  o.s0.re = ((fm * p.s0.re + a * p.s2.re) - c * p.s3.re) - d * p.s3.im;
  o.s0.im = ((fm * p.s0.im + a * p.s2.im) - c * p.s3.im) + d * p.s3.re;
  o.s1.re = ((fm * p.s1.re + b * p.s3.re) - c * p.s2.re) + d * p.s2.im;
  o.s1.im = ((fm * p.s1.im + b * p.s3.im) - c * p.s2.im) - d * p.s2.re;
  o.s2.re = ((fm * p.s2.re + b * p.s0.re) + c * p.s1.re) + d * p.s1.im;
  o.s2.im = ((fm * p.s2.im + b * p.s0.im) + c * p.s1.im) - d * p.s1.re;
  o.s3.re = ((fm * p.s3.re + a * p.s1.re) + c * p.s0.re) - d * p.s0.im;
  o.s3.im = ((fm * p.s3.im + a * p.s1.im) + c * p.s0.im) + d * p.s0.re;
  return o;
}
template <class R> __device__ __forceinline__ void opaque_sp(Sp<R>& p) {
  opaque(p.s0.re);
  opaque(p.s0.im);
  opaque(p.s1.re);
  opaque(p.s1.im);
  opaque(p.s2.re);
  opaque(p.s2.im);
  opaque(p.s3.re);
  opaque(p.s3.im);
}
// Fermion propagator applied to an off-shell spinor: f * (Qslash + m) phi,
// with f folded into the slash coefficients and the mass.
template <class R> __device__ __forceinline__ Sp<R> prop(const V4<R>& Q, R m, R f, const Sp<R>& phi) {
  return pslash(f * m, f * (Q.t - Q.z), f * (Q.t + Q.z), f * Q.x, f * Q.y, phi);
}
// The same for Q = -P: f * (m - Pslash) phi.
template <class R> __device__ __forceinline__ Sp<R> prop_neg(const V4<R>& P, R m, R f, const Sp<R>& phi) {
  const R g = R(0.0) - f;
  return pslash(f * m, g * (P.t - P.z), g * (P.t + P.z), g * P.x, g * P.y, phi);
}
// Row spinor (ubar) times column spinor, real and imaginary parts as single
// chains of fused multiply-adds.
template <class R> __device__ __forceinline__ C2<R> ubar_dot(const Sp<R>& u, const Sp<R>& p) {
  R re = u.s0.re * p.s0.re;
  re = re - u.s0.im * p.s0.im;
  re = re + u.s1.re * p.s1.re;
  re = re - u.s1.im * p.s1.im;
  re = re + u.s2.re * p.s2.re;
  re = re - u.s2.im * p.s2.im;
  re = re + u.s3.re * p.s3.re;
  re = re - u.s3.im * p.s3.im;
  R im = u.s0.re * p.s0.im;
  im = im + u.s0.im * p.s0.re;
  im = im + u.s1.re * p.s1.im;
  im = im + u.s1.im * p.s1.re;
  im = im + u.s2.re * p.s2.im;
  im = im + u.s2.im * p.s2.re;
  im = im + u.s3.re * p.s3.im;
  im = im + u.s3.im * p.s3.re;
  return C2<R>{re, im};
}

// ------------------------------------------------- external wavefunctions
// Two-component helicity eigenstates chi_{+-}(p-hat):
//   chi_+ = (P3, px + i py)/N,  chi_- = (-px + i py, P3)/N,
//   P3 = |p| + pz (evaluated as pT^2/(|p| - pz) for pz < 0), N = sqrt(2|p| P3);
// p along -z: chi_+ = (0, 1), chi_- = (-1, 0).
template <class R> __device__ __forceinline__ void chis(const V4<R>& p, C2<R>* cp, C2<R>* cm) {
  R pt2 = p.x * p.x + p.y * p.y;
  R pp = dsqrt(pt2 + p.z * p.z);
  R P3 = (val(p.z) >= 0) ? pp + p.z : pt2 / (pp - p.z);
  bool minus_z = !(val(P3) > 0);
  R N = dsqrt(R(2.0) * pp * P3);
  R iN = minus_z ? R(0.0) : R(1.0) / N;
  R a = P3 * iN, bx = p.x * iN, by = p.y * iN;
  cp[0] = C2<R>{a, R(0.0)};
  cp[1] = C2<R>{minus_z ? R(1.0) : bx, by};
  cm[0] = C2<R>{minus_z ? R(-1.0) : -bx, by};
  cm[1] = C2<R>{a, R(0.0)};
}
// omega_+- = sqrt(E +- |p|), omega_- evaluated as m / omega_+.
template <class R> __device__ __forceinline__ void omegas(const V4<R>& p, R m, R& wp, R& wm) {
  R pp = dsqrt(p.x * p.x + p.y * p.y + p.z * p.z);
  wp = dsqrt(p.t + pp);
  wm = m / wp;
}
// ubar(p, lambda) for an outgoing fermion: u = (omega_{-l} chi_l ; omega_l chi_l),
// ubar = u^dagger gamma^0 = (u2*, u3*, u0*, u1*).
template <class R> __device__ __forceinline__ Sp<R> ubar_spinor(const V4<R>& p, R m, int lam) {
  C2<R> cp[2], cm[2];
  chis(p, cp, cm);
  R wp, wm;
  omegas(p, m, wp, wm);
  const C2<R>* c = lam > 0 ? cp : cm;
  R lo = lam > 0 ? wm : wp, hi = lam > 0 ? wp : wm;
  Sp<R> u;
  u.s0 = C2<R>{hi * c[0].re, -(hi * c[0].im)};
  u.s1 = C2<R>{hi * c[1].re, -(hi * c[1].im)};
  u.s2 = C2<R>{lo * c[0].re, -(lo * c[0].im)};
  u.s3 = C2<R>{lo * c[1].re, -(lo * c[1].im)};
  return u;
}
// v(p, lambda) for an outgoing antifermion:
//   v = (-l omega_l chi_{-l} ; l omega_{-l} chi_{-l}).
template <class R> __device__ __forceinline__ Sp<R> v_spinor(const V4<R>& p, R m, int lam) {
  C2<R> cp[2], cm[2];
  chis(p, cp, cm);
  R wp, wm;
  omegas(p, m, wp, wm);
  const C2<R>* c = lam > 0 ? cm : cp;
  R wl = lam > 0 ? wp : wm, wml = lam > 0 ? wm : wp;
  R s = R(double(lam));
  R a = -(s * wl), b = s * wml;
  Sp<R> v;
  v.s0 = C2<R>{a * c[0].re, a * c[0].im};
  v.s1 = C2<R>{a * c[1].re, a * c[1].im};
  v.s2 = C2<R>{b * c[0].re, b * c[0].im};
  v.s3 = C2<R>{b * c[1].re, b * c[1].im};
  return v;
}
// The two real linear polarisation vectors of a massless vector boson:
//   e1 = (0, cos t cos f, cos t sin f, -sin t), e2 = (0, -sin f, cos f, 0),
// with f = 0 when the boson moves along the z axis.
template <class R> __device__ __forceinline__ void lin_pols(const V4<R>& k, V4<R>* e) {
  R pt = dsqrt(k.x * k.x + k.y * k.y);
  R kk = dsqrt(k.x * k.x + k.y * k.y + k.z * k.z);
  bool axial = !(val(pt) > 0);
  R ipt = axial ? R(0.0) : R(1.0) / pt;
  R cf = axial ? R(1.0) : k.x * ipt, sf = k.y * ipt;
  R ik = R(1.0) / kk;
  R ct = k.z * ik, st = pt * ik;
  e[0] = V4<R>{R(0.0), ct * cf, ct * sf, -st};
  e[1] = V4<R>{R(0.0), -sf, cf, R(0.0)};
}

}  // namespace mf
