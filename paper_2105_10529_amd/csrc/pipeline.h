// Per-event pipeline stages as device functions (HIP, gfx950): Philox
// uniforms, the VEGAS map, PDF gathers, phase space with cuts, the matrix
// element dispatch and the event weight.  This is the event generation
// pipeline of arXiv:2105.10529 Sec. 2.1 (random numbers -> phase-space
// kinematics -> matrix element), one event per lane, branch-free where the
// lanes of a wavefront would otherwise diverge.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "amp.h"
#include "gen/me_gg_m2.h"
#include "gen/me_gg_m3.h"
#include "gen/me_gg_m4.h"
#include "gen/me_gg_m4_grouped.h"
#include "qq.h"

namespace mf {

constexpr int NXK = 196;        // PDF x knots
constexpr int NQK = 50;         // PDF Q knots
constexpr double PDF_Q0 = 1.65;
constexpr double PDF_QMAX = 1e5;
constexpr double GEV2_PB = 3.893793721e8;
constexpr int MAXD = 13;
constexpr int MAX_BINS = 64;

// Device-side view of one configured process (passed by value).
struct DevCfg {
  int ng;          // final-state gluons
  int channel;     // 0: g g, 1: u u~, 2: d d~
  int ndim;
  int nb;          // VEGAS bins per dimension
  double s;        // hadronic s
  double mt;
  double mu;       // factorisation scale (fixed)
  int mu_is_mt;    // the scale follows m_t in derivatives
  double pt_min, eta_max, dr_min;
  double lx0, ihx;     // ln x of the first knot and inverse knot spacing in ln x
  double norm;     // g^(2m) * (1 / spin-colour average) / n_g! * pb conversion / 2
  const double* pdfc;  // [4][196] x f(x_i, mu), flavours g, u, d, u~
  const double* pdfd;  // [4][196] d(x f)/d mu at x_i
  const double* pdft;  // [8][196] d(x f)/d theta_k at x_i (flavour of theta_k)
  int helicity;        // polarisation-state mode of the staged 5-gluon process (mf_config.helicity)
  uint64_t seed;       // Philox key word 0 (the process seed)
  int dyn_scale;       // 1: factorisation scale mu = H_T / 2 per event
  const double* pdfq;  // [4][50][196] x f(x_i, Q_j) (dynamic scale), else unused
};

// ------------------------------------------------------------------ Philox
// Philox4x64 with 10 rounds (Salmon et al., SC'11); counter (c0..c3), key (k0,k1).
struct U4 {
  uint64_t x0, x1, x2, x3;
};
__device__ __forceinline__ U4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                            uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return U4{c0, c1, c2, c3};
}
__device__ __forceinline__ double u01(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1.0p-53; }

// ndim uniforms of event ev: counter (ev, iter, call, 0), key (seed, purpose).
__device__ __forceinline__ void event_uniforms(uint64_t ev, uint64_t iter, uint64_t seed, uint64_t purpose,
                                               int d, double* u) {
#pragma unroll
  for (int call = 0; call < (MAXD + 3) / 4; ++call) {
    if (call * 4 < d) {
      U4 r = philox4x64_10(ev, iter, (uint64_t)call, 0, seed, purpose);
      u[call * 4 + 0] = u01(r.x0);
      if (call * 4 + 1 < MAXD) u[call * 4 + 1] = u01(r.x1);
      if (call * 4 + 2 < MAXD) u[call * 4 + 2] = u01(r.x2);
      if (call * 4 + 3 < MAXD) u[call * 4 + 3] = u01(r.x3);
    }
  }
}

// ------------------------------------------------------------------- VEGAS
// y -> x through the adaptive bins of one dimension (edges e[0..nb]).
__device__ __forceinline__ double vegas_map_dim(const double* e, int nb, double y, int& bin, double& jac) {
  double t = y * nb;
  int k = (int)floor(t);
  k = k < 0 ? 0 : (k >= nb ? nb - 1 : k);
  double lo = e[k], wdt = e[k + 1] - lo;
  bin = k;
  jac *= nb * wdt;
  return lo + (t - k) * wdt;
}

// -------------------------------------------------------------------- PDFs
// Cubic Hermite on the 196 x knots (unit spacing in t) with central-difference
// slopes, one-sided at the two end knots; returns the value at t.
__device__ __forceinline__ double hermite_x(const double* f, double t) {
  int i = (int)floor(t);
  i = i < 0 ? 0 : (i > NXK - 2 ? NXK - 2 : i);
  double u = t - i;
  double fm = f[i > 0 ? i - 1 : 0], f0 = f[i], f1 = f[i + 1], f2 = f[i + 2 < NXK ? i + 2 : NXK - 1];
  double s0 = (i == 0) ? f1 - f0 : 0.5 * (f1 - fm);
  double s1 = (i + 1 == NXK - 1) ? f1 - f0 : 0.5 * (f2 - f0);
  double u2 = u * u, u3 = u2 * u;
  double h00 = 2.0 * u3 - 3.0 * u2 + 1.0, h10 = u3 - 2.0 * u2 + u, h01 = -2.0 * u3 + 3.0 * u2, h11 = u3 - u2;
  return h00 * f0 + h10 * s0 + h01 * f1 + h11 * s1;
}
__device__ __forceinline__ double x_position(const DevCfg& c, double x) { return (log(x) - c.lx0) * c.ihx; }

// Dynamic scale: mu = H_T / 2, half the sum of the final-state transverse
// masses (tops of mass m_t, massless gluons), and x f(x, mu) from the full
// knot table by the same tensor-product Hermite scheme as the fixed-scale
// tables (along x on the four Q rows around mu, then along Q).
template <int NG, class RK>
__device__ __forceinline__ double half_ht(double mt, const V4<RK>& top, const V4<RK>& atop, const V4<double>* gl) {
  const double tx = val(top.x), ty = val(top.y), ax = val(atop.x), ay = val(atop.y);
  double ht = sqrt(mt * mt + tx * tx + ty * ty) + sqrt(mt * mt + ax * ax + ay * ay);
#pragma unroll
  for (int i = 0; i < NG; ++i) ht += sqrt(gl[i].x * gl[i].x + gl[i].y * gl[i].y);
  return 0.5 * ht;
}
__device__ __forceinline__ double q_position(double mu) {
  return (log(mu) - log(PDF_Q0)) / ((log(PDF_QMAX) - log(PDF_Q0)) / (NQK - 1));
}
__device__ __forceinline__ double hermite_xq(const double* tab, double tx, double tq) {
  int j = (int)floor(tq);
  j = j < 0 ? 0 : (j > NQK - 2 ? NQK - 2 : j);
  const double u = tq - j;
  double F[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int jj = j - 1 + r;
    jj = jj < 0 ? 0 : (jj > NQK - 1 ? NQK - 1 : jj);
    F[r] = hermite_x(tab + (int64_t)jj * NXK, tx);
  }
  const double s0 = (j == 0) ? F[2] - F[1] : 0.5 * (F[2] - F[0]);
  const double s1 = (j + 1 == NQK - 1) ? F[2] - F[1] : 0.5 * (F[3] - F[1]);
  const double u2 = u * u, u3 = u2 * u;
  return (2.0 * u3 - 3.0 * u2 + 1.0) * F[1] + (u3 - 2.0 * u2 + u) * s0 + (-2.0 * u3 + 3.0 * u2) * F[2] +
         (u3 - u2) * s1;
}
// x f of flavour fl at x-table position t: from the fixed-scale tables pdf1
// ([4][196]) or, with the dynamic scale, from the full table at Q position tq
__device__ __forceinline__ double pdf_at(const DevCfg& c, const double* pdf1, int fl, double t, double tq) {
  return c.dyn_scale ? hermite_xq(c.pdfq + (int64_t)fl * NQK * NXK, t, tq) : hermite_x(pdf1 + fl * NXK, t);
}

// ------------------------------------------------------------ phase space
template <class R>
__device__ __forceinline__ V4<R> boost_from_rest(const V4<R>& p, const V4<R>& Q, R M) {
  R bp = Q.x * p.x + Q.y * p.y + Q.z * p.z;
  R iM = R(1.0) / M;
  R e = (Q.t * p.t + bp) * iM;
  R c = (bp / (Q.t + M) + p.t) * iM;
  return V4<R>{e, p.x + c * Q.x, p.y + c * Q.y, p.z + c * Q.z};
}

// v^k for a small non-negative integer k, by multiplication (the exponents
// here are at most the number of final-state bodies)
__device__ __forceinline__ double ipow(double v, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= v;
  return r;
}

// Solve (N-1) v^(N-2) - (N-2) v^(N-1) = r on [0,1] (the distribution of
// v = M_i^2/M_{i-1}^2 for N massless bodies): closed form for N = 3,
// otherwise bisection to 2^-40 then safeguarded Newton steps.  The
// polynomial is evaluated as v^(N-3) (v ((N-1) - (N-2) v)) with integer
// powers.
__device__ __forceinline__ double solve_mass_ratio(int N, double r) {
  if (N == 3) return r / (1.0 + sqrt(1.0 - r));
  double lo = 0.0, hi = 1.0;
  const double a = N - 1, b = N - 2;
  for (int it = 0; it < 40; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double F = ipow(mid, N - 2) * (a - b * mid);
    if (F < r) lo = mid; else hi = mid;
  }
  double v = 0.5 * (lo + hi);
  for (int it = 0; it < 4; ++it) {
    const double p3 = ipow(v, N - 3);
    const double F = p3 * v * (a - b * v) - r;
    const double dF = a * b * p3 * (1.0 - v);
    const double nv = dF > 0.0 ? v - F / dF : v;
    v = (nv > lo && nv < hi) ? nv : v;
  }
  return v;
}

// Final state from x[2..] in the partonic centre-of-mass frame: the gluons
// are emitted one by one from the massless n-body recursion (Platzer,
// "RAMBO on diet"), the top pair is split last; returns V_n(s) * beta or 0
// below threshold.  Gluon momenta do not depend on m_t.
template <class R>
__device__ __forceinline__ R phase_space(int ng, const double* x, double shat, R mt, V4<double>* gl, V4<R>& top,
                                         V4<R>& atop) {
  const int n = ng + 2;
  double M = sqrt(shat);
  V4<double> Q{M, 0.0, 0.0, 0.0};
  double Mprev = M;
  for (int i = 1; i <= n - 2; ++i) {
    double v = solve_mass_ratio(n - i + 1, x[2 + (i - 1)]);
    double Mi = Mprev * sqrt(v);
    double q = (Mprev * Mprev - Mi * Mi) / (2.0 * Mprev);
    double ct = 2.0 * x[2 + (n - 2) + 2 * (i - 1)] - 1.0;
    double ph = 2.0 * M_PI * x[2 + (n - 2) + 2 * (i - 1) + 1];
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double sp, cp;
    sincos(ph, &sp, &cp);
    V4<double> g{q, q * st * cp, q * st * sp, q * ct};
    V4<double> rest{sqrt(Mi * Mi + q * q), -g.x, -g.y, -g.z};
    gl[i - 1] = boost_from_rest(g, Q, Mprev);
    Q = boost_from_rest(rest, Q, Mprev);
    Mprev = Mi;
  }
  // t t~ split of the remaining system of mass Mprev.  Below threshold the
  // kinematics are built for a safe mass just above it and the weight is 0,
  // so every lane follows the same instruction stream.
  const bool above = Mprev > 2.0 * val(mt);
  R Mtt = above ? R(Mprev) : R(2.0) * mt * R(1.0 + 1e-6);
  R beta = dsqrt(R(1.0) - R(4.0) * mt * mt / (Mtt * Mtt));
  R q = Mtt * beta * R(0.5);
  double ct = 2.0 * x[2 + (n - 2) + 2 * (n - 2)] - 1.0;
  double ph = 2.0 * M_PI * x[2 + (n - 2) + 2 * (n - 2) + 1];
  double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  double sp, cp;
  sincos(ph, &sp, &cp);
  R E = Mtt * R(0.5);
  V4<R> t{E, q * R(st * cp), q * R(st * sp), q * R(ct)};
  V4<R> tb{E, R(0.0) - t.x, R(0.0) - t.y, R(0.0) - t.z};
  // rest frame of the pair: its momentum Q with the (possibly safe) mass Mtt
  V4<R> QR{above ? R(Q.t) : dsqrt(Mtt * Mtt + R(Q.x * Q.x + Q.y * Q.y + Q.z * Q.z)), R(Q.x), R(Q.y), R(Q.z)};
  top = boost_from_rest(t, QR, Mtt);
  atop = boost_from_rest(tb, QR, Mtt);
  // massless volume V_n(s) = (2 pi)^(4-3n) (pi/2)^(n-1) s^(n-2) / ((n-1)! (n-2)!)
  double vol = pow(2.0 * M_PI, 4.0 - 3.0 * n) * pow(0.5 * M_PI, n - 1.0) * ipow(shat, n - 2);
  double fact = 1.0;
  for (int k = 2; k <= n - 1; ++k) fact *= k;
  double fact2 = 1.0;
  for (int k = 2; k <= n - 2; ++k) fact2 *= k;
  return above ? R(vol / (fact * fact2)) * beta : R(0.0);
}

// Fiducial cuts on the gluons in the lab frame: the lab rapidity differs from
// the centre-of-mass one by y = ln(x1/x2)/2; pT and azimuths are invariant.
__device__ __forceinline__ bool pass_cuts(const DevCfg& c, int ng, const V4<double>* g, double yboost) {
  double eta[3], phi[3];
  bool ok = true;
  for (int i = 0; i < ng; ++i) {
    double pt = sqrt(g[i].x * g[i].x + g[i].y * g[i].y);
    double pp = sqrt(pt * pt + g[i].z * g[i].z);
    eta[i] = atanh(g[i].z / pp) + yboost;
    phi[i] = atan2(g[i].y, g[i].x);
    ok = ok && (pt > c.pt_min) && (fabs(eta[i]) < c.eta_max);
  }
  if (c.dr_min > 0.0)
    for (int i = 0; i < ng; ++i)
      for (int j = i + 1; j < ng; ++j) {
        double dphi = fabs(phi[i] - phi[j]);
        dphi = dphi > M_PI ? 2.0 * M_PI - dphi : dphi;
        double de = eta[i] - eta[j];
        ok = ok && (sqrt(de * de + dphi * dphi) > c.dr_min);
      }
  return ok;
}

// ------------------------------------------------------ matrix elements
template <class RA, class RK> __device__ __forceinline__ V4<RA> to_amp(const V4<RK>& p);
template <> __device__ __forceinline__ V4<double> to_amp<double, double>(const V4<double>& p) { return p; }
template <> __device__ __forceinline__ V4<float> to_amp<float, double>(const V4<double>& p) {
  return V4<float>{(float)p.t, (float)p.x, (float)p.y, (float)p.z};
}
template <> __device__ __forceinline__ V4<Dual<double>> to_amp<Dual<double>, Dual<double>>(const V4<Dual<double>>& p) {
  return p;
}
template <> __device__ __forceinline__ V4<Dual<float>> to_amp<Dual<float>, Dual<double>>(const V4<Dual<double>>& p) {
  return V4<Dual<float>>{Dual<float>((float)p.t.v, (float)p.t.d), Dual<float>((float)p.x.v, (float)p.x.d),
                         Dual<float>((float)p.y.v, (float)p.y.d), Dual<float>((float)p.z.v, (float)p.z.d)};
}
template <> __device__ __forceinline__ V4<Dual<double>> to_amp<Dual<double>, double>(const V4<double>& p) {
  return V4<Dual<double>>{Dual<double>(p.t), Dual<double>(p.x), Dual<double>(p.y), Dual<double>(p.z)};
}
template <> __device__ __forceinline__ V4<Dual<float>> to_amp<Dual<float>, double>(const V4<double>& p) {
  return V4<Dual<float>>{Dual<float>((float)p.t), Dual<float>((float)p.x), Dual<float>((float)p.y),
                         Dual<float>((float)p.z)};
}
__device__ __forceinline__ double to_amp_s(double x, double*) { return x; }
__device__ __forceinline__ float to_amp_s(double x, float*) { return (float)x; }
__device__ __forceinline__ Dual<double> to_amp_s(Dual<double> x, Dual<double>*) { return x; }
__device__ __forceinline__ Dual<float> to_amp_s(Dual<double> x, Dual<float>*) { return Dual<float>((float)x.v, (float)x.d); }

// Colour- and polarisation-summed |M|^2 (g = 1) for g g -> t t~ + NG g.
// E: beam energy; gluons in emission order; top/atop from the phase space.
// Momenta and per-event invariants stay in the kinematic type RK; the
// helicity loops run in the amplitude type RA.
template <int NG, class RA, class RK>
__device__ __forceinline__ RA me_gg(double E, const V4<double>* gl, const V4<RK>& top, const V4<RK>& atop, RK mt) {
  constexpr int m = NG + 2;
  V4<RK> K[m];
  V4<RA> Ep[m][2];
  K[0] = V4<RK>{RK(-E), RK(0.0), RK(0.0), RK(-E)};
  K[1] = V4<RK>{RK(-E), RK(0.0), RK(0.0), RK(E)};
  const RA z = RA(0.0), o = RA(1.0);
  Ep[0][0] = V4<RA>{z, o, z, z};
  Ep[0][1] = V4<RA>{z, z, o, z};
  Ep[1][0] = V4<RA>{z, o, z, z};
  Ep[1][1] = V4<RA>{z, z, o, z};
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    K[2 + i] = V4<RK>{RK(gl[i].t), RK(gl[i].x), RK(gl[i].y), RK(gl[i].z)};
    lin_pols(cvt4<RA>(K[2 + i]), Ep[2 + i]);
  }
  RA m_a = cvt<RA>(mt);
  V4<RA> t = cvt4<RA>(top), tb = cvt4<RA>(atop);
  Sp<RA> UB[2] = {ubar_spinor(t, m_a, -1), ubar_spinor(t, m_a, 1)};
  Sp<RA> VS[2] = {v_spinor(tb, m_a, -1), v_spinor(tb, m_a, 1)};
  if constexpr (m == 2) return me_gg_m2<RA, RK>(K, Ep, UB, VS, atop, mt);
  else if constexpr (m == 3) return me_gg_m3<RA, RK>(K, Ep, UB, VS, atop, mt);
  else if constexpr (std::is_same<RA, float>::value) return me_gg_m4_grouped<RA, RK>(K, Ep, UB, VS, atop, mt);
  else return me_gg_m4<RA, RK>(K, Ep, UB, VS, atop, mt);
}

// Row spinor psibar gamma^mu chi contracted: returns the four components
// of the current psibar gamma^mu chi (contravariant).
template <class R> __device__ __forceinline__ void vcurrent(const Sp<R>& r, const Sp<R>& c, C2<R>* j) {
  // gamma^mu = [[0, sigma^mu], [sigmabar^mu, 0]], sigma = (1, s), sigmabar = (1, -s)
  j[0] = cmul(r.s0, c.s2) + cmul(r.s1, c.s3) + cmul(r.s2, c.s0) + cmul(r.s3, c.s1);
  // sigma_x: r0 c3 + r1 c2 ;  -(r2 c1 + r3 c0)
  j[1] = (cmul(r.s0, c.s3) + cmul(r.s1, c.s2)) - (cmul(r.s2, c.s1) + cmul(r.s3, c.s0));
  // sigma_y: -i r0 c3 + i r1 c2 ;  -(-i r2 c1 + i r3 c0)
  C2<R> a = cmul(r.s1, c.s2) - cmul(r.s0, c.s3);  // times i
  C2<R> b = cmul(r.s2, c.s1) - cmul(r.s3, c.s0);  // times i
  C2<R> ab = a + b;
  j[2] = C2<R>{R(0.0) - ab.im, ab.re};
  // sigma_z: r0 c2 - r1 c3 ; -(r2 c0 - r3 c1)
  j[3] = (cmul(r.s0, c.s2) - cmul(r.s1, c.s3)) - (cmul(r.s2, c.s0) - cmul(r.s3, c.s1));
}
// psibar from a column spinor: psi^dagger gamma^0 = (p2*, p3*, p0*, p1*)
template <class R> __device__ __forceinline__ Sp<R> dbar(const Sp<R>& p) {
  return Sp<R>{C2<R>{p.s2.re, R(0.0) - p.s2.im}, C2<R>{p.s3.re, R(0.0) - p.s3.im},
               C2<R>{p.s0.re, R(0.0) - p.s0.im}, C2<R>{p.s1.re, R(0.0) - p.s1.im}};
}
template <class R> __device__ __forceinline__ Sp<R> u_spinor(const V4<R>& p, R m, int lam) {
  return dbar(ubar_spinor(p, m, lam));
}

// q(p1) q~(p2) -> t t~: colour- and helicity-summed |M|^2 (g = 1) of the
// s-channel gluon diagram; colour factor sum Tr(t^a t^b)^2 = 2.
template <class RA, class RK>
__device__ __forceinline__ RA me_qqbar(const V4<double>& p1, const V4<double>& p2, const V4<RK>& top,
                                       const V4<RK>& atop, RK mt) {
  V4<RA> a = to_amp<RA, double>(p1), b = to_amp<RA, double>(p2);
  V4<RA> t = to_amp<RA, RK>(top), tb = to_amp<RA, RK>(atop);
  RA m_a = to_amp_s(mt, (RA*)nullptr);
  RA z = RA(0.0);
  V4<RA> P = a + b;
  RA sh = mdot(P, P);
  RA tot = RA(0.0);
#pragma unroll 1
  for (int h = 0; h < 16; ++h) {
    int l1 = (h & 8) ? 1 : -1, l2 = (h & 4) ? 1 : -1, l3 = (h & 2) ? 1 : -1, l4 = (h & 1) ? 1 : -1;
    Sp<RA> u1 = u_spinor(a, z, l1);
    Sp<RA> vb2 = dbar(v_spinor(b, z, l2));
    Sp<RA> ub3 = ubar_spinor(t, m_a, l3);
    Sp<RA> v4 = v_spinor(tb, m_a, l4);
    C2<RA> ji[4], jo[4];
    vcurrent(vb2, u1, ji);
    vcurrent(ub3, v4, jo);
    C2<RA> amp = cmul(jo[0], ji[0]) - cmul(jo[1], ji[1]) - cmul(jo[2], ji[2]) - cmul(jo[3], ji[3]);
    tot = tot + cabs2(amp);
  }
  return RA(2.0) * tot / (sh * sh);
}

// --------------------------------------------------------- event weight
// Amplitude-precision result converted back to the kinematic type.
__device__ __forceinline__ double to_k(double a, double*) { return a; }
__device__ __forceinline__ double to_k(float a, double*) { return (double)a; }
__device__ __forceinline__ Dual<double> to_k(Dual<double> a, Dual<double>*) { return a; }
__device__ __forceinline__ Dual<double> to_k(Dual<float> a, Dual<double>*) {
  return Dual<double>((double)a.v, (double)a.d);
}

// Result of one event.  w = r1 * f(x1) f(x2) for g g; for q q~,
// w = r1 q(x1) q~(x2) + r2 q~(x1) q(x2).  r1, r2 hold every factor but the
// PDFs (they carry the m_t derivative in the dual case).
template <class R> struct EventOut {
  R w, r1, r2, r3, r4;
  double t1, t2;  // PDF table positions of x1, x2
  int pass;
};

// Whether the event at x has kinematics and passes the cuts: the same
// decision, in the same FP64 arithmetic, as the selection of event_weight
// with the kinematic type double.
template <int NG>
__device__ __forceinline__ bool event_passes(const DevCfg& c, const double* x) {
  const double x1 = x[0], x2 = x[1];
  const double shat = x1 * x2 * c.s;
  const double thr = 4.0 * c.mt * c.mt;
  bool ok = shat > thr;
  const double shat_k = ok ? shat : thr * (1.0 + 1e-3);
  V4<double> gl[NG > 0 ? NG : 1];
  V4<double> top, atop;
  const double wps = phase_space<double>(NG, x, shat_k, c.mt, gl, top, atop);
  ok = ok && (wps > 0.0);
  return ok && pass_cuts(c, NG, gl, 0.5 * log(x1 / x2));
}

// The integrand at x (unit hypercube, after the VEGAS map).  Branch-free:
// an event below threshold or outside the cuts is evaluated on safe
// kinematics and its weight is selected to zero, so the amplitude code never
// runs under a partial execution mask.
template <int NG, int CH, class RA, class RK>
__device__ __forceinline__ EventOut<RK> event_weight(const DevCfg& c, const double* x, RK mt, const double* pdf) {
  EventOut<RK> out;
  double x1 = x[0], x2 = x[1];
  double shat = x1 * x2 * c.s;
  const double thr = 4.0 * val(mt) * val(mt);
  bool ok = shat > thr;
  const double shat_k = ok ? shat : thr * (1.0 + 1e-3);
  V4<double> gl[NG > 0 ? NG : 1];
  V4<RK> top, atop;
  RK wps = phase_space<RK>(NG, x, shat_k, mt, gl, top, atop);
  ok = ok && (val(wps) > 0.0);
  ok = ok && pass_cuts(c, NG, gl, 0.5 * log(x1 / x2));
  out.pass = ok ? 1 : 0;
  double E = 0.5 * sqrt(shat_k);
  out.t1 = x_position(c, x1);
  out.t2 = x_position(c, x2);
  RK pre = RK(c.norm / (2.0 * shat_k * x1 * x2)) * wps;
  const RK zero = RK(0.0);
  const double tq = c.dyn_scale ? q_position(half_ht<NG>(val(mt), top, atop, gl)) : 0.0;
  if constexpr (CH == 0) {
    RK me = to_k(me_gg<NG, RA, RK>(E, gl, top, atop, mt), (RK*)nullptr);
    RK r1 = pre * me;
    RK w = r1 * RK(pdf_at(c, pdf, 0, out.t1, tq) * pdf_at(c, pdf, 0, out.t2, tq));
    out.r1 = ok ? r1 : zero;
    out.r2 = zero;
    out.r3 = zero;
    out.r4 = zero;
    out.w = ok ? w : zero;
  } else if constexpr (NG == 0 || CH != 3) {
    // q q~ -> t t~ (+ g): the quark from beam 1 (r1) or from beam 2 (r2)
    V4<double> p1{E, 0.0, 0.0, E}, p2{E, 0.0, 0.0, -E};
    RK r1, r2;
    if constexpr (NG == 0) {
      r1 = pre * to_k(me_qqbar<RA, RK>(p1, p2, top, atop, mt), (RK*)nullptr);
      r2 = pre * to_k(me_qqbar<RA, RK>(p2, p1, top, atop, mt), (RK*)nullptr);
    } else {
      const V4<RA> a = to_amp<RA, double>(p1), b = to_amp<RA, double>(p2), k = to_amp<RA, double>(gl[0]);
      const V4<RA> t = to_amp<RA, RK>(top), tb = to_amp<RA, RK>(atop);
      const RA m_a = to_amp_s(mt, (RA*)nullptr);
      // one copy of the matrix-element code for both beam assignments
      r1 = r2 = zero;
#pragma unroll 1
      for (int j = 0; j < 2; ++j) {
        const RK rj = pre * to_k(me_qqbar_g<RA>(j ? b : a, j ? a : b, t, tb, k, m_a), (RK*)nullptr);
        r1 = j ? r1 : rj;
        r2 = j ? rj : r2;
      }
    }
    const int fq = CH == 1 ? 1 : 2, fa = 3;
    double q1 = pdf_at(c, pdf, fq, out.t1, tq), a2 = pdf_at(c, pdf, fa, out.t2, tq),
           a1 = pdf_at(c, pdf, fa, out.t1, tq), q2 = pdf_at(c, pdf, fq, out.t2, tq);
    RK w = r1 * RK(q1 * a2) + r2 * RK(a1 * q2);
    out.r1 = ok ? r1 : zero;
    out.r2 = ok ? r2 : zero;
    out.r3 = zero;
    out.r4 = zero;
    out.w = ok ? w : zero;
  } else {
    // q g -> t t~ q (q = u, d) from either beam (r1: quark from beam 1, r2:
    // from beam 2) and q~ g -> t t~ q~ (q~ = u~, d~, equal PDFs): by charge
    // conjugation its |M|^2 is that of q g -> t t~ q with the top and
    // antitop momenta exchanged (r3: antiquark from beam 1, r4: from beam 2)
    V4<double> p1{E, 0.0, 0.0, E}, p2{E, 0.0, 0.0, -E};
    const V4<RA> a = to_amp<RA, double>(p1), b = to_amp<RA, double>(p2), k = to_amp<RA, double>(gl[0]);
    const V4<RA> t = to_amp<RA, RK>(top), tb = to_amp<RA, RK>(atop);
    const RA m_a = to_amp_s(mt, (RA*)nullptr);
    // one copy of the matrix-element code for the four assignments
    RK r1 = zero, r2 = zero, r3 = zero, r4 = zero;
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
      const bool sw = (j & 1) != 0, cc = (j & 2) != 0;
      const RK rj = pre * to_k(me_qg_q<RA>(sw ? b : a, sw ? a : b, cc ? tb : t, cc ? t : tb, k, m_a), (RK*)nullptr);
      r1 = j == 0 ? rj : r1;
      r2 = j == 1 ? rj : r2;
      r3 = j == 2 ? rj : r3;
      r4 = j == 3 ? rj : r4;
    }
    const double g1 = pdf_at(c, pdf, 0, out.t1, tq), g2 = pdf_at(c, pdf, 0, out.t2, tq);
    const double qs1 = pdf_at(c, pdf, 1, out.t1, tq) + pdf_at(c, pdf, 2, out.t1, tq);
    const double qs2 = pdf_at(c, pdf, 1, out.t2, tq) + pdf_at(c, pdf, 2, out.t2, tq);
    const double as1 = 2.0 * pdf_at(c, pdf, 3, out.t1, tq), as2 = 2.0 * pdf_at(c, pdf, 3, out.t2, tq);
    RK w = r1 * RK(qs1 * g2) + r2 * RK(g1 * qs2) + r3 * RK(as1 * g2) + r4 * RK(g1 * as2);
    out.r1 = ok ? r1 : zero;
    out.r2 = ok ? r2 : zero;
    out.r3 = ok ? r3 : zero;
    out.r4 = ok ? r4 : zero;
    out.w = ok ? w : zero;
  }
  return out;
}

}  // namespace mf
