// Plain FP64 CPU oracle for the per-event leading-order integrand of a
// parton-level Monte Carlo (arXiv:2105.10529).
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library links, includes or
// calls this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark load the shared object built from it. It shares no code,
// header, table or constant generator with the HIP path.
//
// What it computes, in the order of the event pipeline of Sec. 2.1 (random
// numbers -> phase-space kinematics -> matrix element -> histogram
// accumulation), written for clarity, not speed:
//   * Philox4x64-10 counter-based generator (Salmon et al., SC'11).
//   * VEGAS importance map, grid refinement and iteration combination
//     (Lepage, J. Comput. Phys. 27 (1978) 192).
//   * Synthetic PDFs on a (ln x, ln Q) grid with tensor-product cubic
//     Hermite ("log-bicubic") interpolation (the PDF ingredient of Sec. 1).
//   * n-body phase space: the massless recursion of Platzer
//     (arXiv:1308.2922, "RAMBO on diet") with the gluons emitted first and the
//     massive top pair split last; fiducial cuts (Sec. 1, third ingredient).
//   * Tree-level |M|^2 for g g -> t t~ + n gluons from helicity wavefunctions
//     and vertices (Sec. 2.2: loop over helicities, aggregate), as
//     colour-ordered Berends-Giele currents contracted with a colour matrix,
//     and q q~ -> t t~ by its single diagram.
//   * Forward-mode dual numbers for derivatives in m_t and PDF parameters.
//
// Conventions: metric (+,-,-,-); chiral Dirac matrices; Tr(t^a t^b) = delta/2;
// all momenta outgoing inside the recursion; the coupling g is set to 1 in
// the recursion and restored as g^(2m) on |M|^2.

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

using std::exp;
using std::log;
using std::pow;
using std::sqrt;

// ---------------------------------------------------------------- dual numbers
struct Dual {
  double v, d;
  Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, s > 0 ? a.d / (2.0 * s) : 0.0);
}
inline Dual log(Dual a) { return Dual(std::log(a.v), a.d / a.v); }
inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
inline Dual pow(Dual a, Dual b) { return exp(b * log(a)); }
inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }
inline double der(double) { return 0.0; }
inline double der(Dual x) { return x.d; }

// -------------------------------------------------------------------- complex
template <class R> struct Cx {
  R re, im;
  Cx(R r = R(0.0), R i = R(0.0)) : re(r), im(i) {}
};
template <class R> inline Cx<R> operator+(Cx<R> a, Cx<R> b) { return Cx<R>(a.re + b.re, a.im + b.im); }
template <class R> inline Cx<R> operator-(Cx<R> a, Cx<R> b) { return Cx<R>(a.re - b.re, a.im - b.im); }
template <class R> inline Cx<R> operator-(Cx<R> a) { return Cx<R>(-a.re, -a.im); }
template <class R> inline Cx<R> operator*(Cx<R> a, Cx<R> b) {
  return Cx<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class R> inline Cx<R> scale(Cx<R> a, R s) { return Cx<R>(a.re * s, a.im * s); }
template <class R> inline Cx<R> conj(Cx<R> a) { return Cx<R>(a.re, -a.im); }

template <class R> using CV = Cx<R>[4];  // complex four-vector or Dirac spinor

// Real four-vectors.
template <class R> struct P4 {
  R e, x, y, z;
};
template <class R> inline R mdot(const P4<R>& a, const P4<R>& b) {
  return a.e * b.e - a.x * b.x - a.y * b.y - a.z * b.z;
}

// Complex four-vector / spinor as a small struct so it can be copied.
template <class R> struct C4 {
  Cx<R> c[4];
};
template <class R> inline C4<R> c4zero() {
  C4<R> r;
  for (int i = 0; i < 4; ++i) r.c[i] = Cx<R>();
  return r;
}
// Minkowski bilinear product of complex four-vectors (no conjugation).
template <class R> inline Cx<R> cdot(const C4<R>& a, const C4<R>& b) {
  return a.c[0] * b.c[0] - a.c[1] * b.c[1] - a.c[2] * b.c[2] - a.c[3] * b.c[3];
}
template <class R> inline C4<R> c4add(const C4<R>& a, const C4<R>& b) {
  C4<R> r;
  for (int i = 0; i < 4; ++i) r.c[i] = a.c[i] + b.c[i];
  return r;
}
template <class R> inline C4<R> c4scale(const C4<R>& a, Cx<R> s) {
  C4<R> r;
  for (int i = 0; i < 4; ++i) r.c[i] = a.c[i] * s;
  return r;
}
template <class R> inline C4<R> fromP4(const P4<R>& p) {
  C4<R> r;
  r.c[0] = Cx<R>(p.e);
  r.c[1] = Cx<R>(p.x);
  r.c[2] = Cx<R>(p.y);
  r.c[3] = Cx<R>(p.z);
  return r;
}

// ------------------------------------------------------------ Dirac matrices
// Chiral representation: gamma^0 = [[0,1],[1,0]], gamma^k = [[0,s^k],[-s^k,0]].
struct Gam {
  double re[4][4][4], im[4][4][4];  // [mu][row][col]
  Gam() {
    std::memset(re, 0, sizeof(re));
    std::memset(im, 0, sizeof(im));
    // Pauli matrices
    double sr[3][2][2] = {{{0, 1}, {1, 0}}, {{0, 0}, {0, 0}}, {{1, 0}, {0, -1}}};
    double si[3][2][2] = {{{0, 0}, {0, 0}}, {{0, -1}, {1, 0}}, {{0, 0}, {0, 0}}};
    for (int a = 0; a < 2; ++a) {
      re[0][a][a + 2] = 1.0;
      re[0][a + 2][a] = 1.0;
    }
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          re[k + 1][a][b + 2] = sr[k][a][b];
          im[k + 1][a][b + 2] = si[k][a][b];
          re[k + 1][a + 2][b] = -sr[k][a][b];
          im[k + 1][a + 2][b] = -si[k][a][b];
        }
  }
};
static const Gam GAM;
static const double METRIC[4] = {1.0, -1.0, -1.0, -1.0};

template <class R> struct M4 {
  Cx<R> a[4][4];
};
// slash(J) = gamma^mu J_mu = sum_mu g_{mu mu} J^mu gamma^mu
template <class R> inline M4<R> slash(const C4<R>& J) {
  M4<R> m;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      Cx<R> s;
      for (int mu = 0; mu < 4; ++mu) {
        Cx<R> g(R(GAM.re[mu][r][c] * METRIC[mu]), R(GAM.im[mu][r][c] * METRIC[mu]));
        s = s + g * J.c[mu];
      }
      m.a[r][c] = s;
    }
  return m;
}
template <class R> inline C4<R> matvec(const M4<R>& m, const C4<R>& v) {
  C4<R> r;
  for (int i = 0; i < 4; ++i) {
    Cx<R> s;
    for (int j = 0; j < 4; ++j) s = s + m.a[i][j] * v.c[j];
    r.c[i] = s;
  }
  return r;
}
template <class R> inline C4<R> rowmat(const C4<R>& row, const M4<R>& m) {
  C4<R> r;
  for (int j = 0; j < 4; ++j) {
    Cx<R> s;
    for (int i = 0; i < 4; ++i) s = s + row.c[i] * m.a[i][j];
    r.c[j] = s;
  }
  return r;
}
template <class R> inline Cx<R> rowvec(const C4<R>& row, const C4<R>& v) {
  Cx<R> s;
  for (int i = 0; i < 4; ++i) s = s + row.c[i] * v.c[i];
  return s;
}
// Dirac adjoint: psibar = psi^dagger gamma^0
template <class R> inline C4<R> dbar(const C4<R>& psi) {
  C4<R> r;
  for (int j = 0; j < 4; ++j) {
    Cx<R> s;
    for (int i = 0; i < 4; ++i) s = s + conj(psi.c[i]) * Cx<R>(R(GAM.re[0][i][j]), R(GAM.im[0][i][j]));
    r.c[j] = s;
  }
  return r;
}

// ------------------------------------------------------- external wavefunctions
// Two-component helicity eigenstates chi_lambda(p-hat) with lambda = +-1
// (HELAS phase conventions; p along -z handled explicitly).
template <class R> inline void chi(const P4<R>& p, int lam, Cx<R> out[2]) {
  R pp = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
  R a = pp + p.z;
  if (val(a) <= 1e-300 * (1.0 + val(pp))) {
    if (lam > 0) { out[0] = Cx<R>(); out[1] = Cx<R>(R(1.0)); }
    else { out[0] = Cx<R>(R(-1.0)); out[1] = Cx<R>(); }
    return;
  }
  R nrm = sqrt(R(2.0) * pp * a);
  if (lam > 0) {
    out[0] = Cx<R>(a / nrm);
    out[1] = Cx<R>(p.x / nrm, p.y / nrm);
  } else {
    out[0] = Cx<R>(-p.x / nrm, p.y / nrm);
    out[1] = Cx<R>(a / nrm);
  }
}
// omega_+ = sqrt(E+|p|), omega_- = sqrt(E-|p|) = m / omega_+
template <class R> inline void omegas(const P4<R>& p, R m, R& wp, R& wm) {
  R pp = sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
  wp = sqrt(p.e + pp);
  wm = (val(m) == 0.0) ? R(0.0) : m / wp;
}
// u(p, lambda) = [omega_{-lambda} chi_lambda ; omega_lambda chi_lambda]
template <class R> inline C4<R> uspinor(const P4<R>& p, R m, int lam) {
  R wp, wm;
  omegas(p, m, wp, wm);
  Cx<R> c[2];
  chi(p, lam, c);
  R wlo = lam > 0 ? wm : wp;  // omega_{-lambda}
  R whi = lam > 0 ? wp : wm;  // omega_{lambda}
  C4<R> u;
  u.c[0] = scale(c[0], wlo);
  u.c[1] = scale(c[1], wlo);
  u.c[2] = scale(c[0], whi);
  u.c[3] = scale(c[1], whi);
  return u;
}
// v(p, lambda) = [-lambda omega_lambda chi_{-lambda} ; lambda omega_{-lambda} chi_{-lambda}]
template <class R> inline C4<R> vspinor(const P4<R>& p, R m, int lam) {
  R wp, wm;
  omegas(p, m, wp, wm);
  Cx<R> c[2];
  chi(p, -lam, c);
  R wl = lam > 0 ? wp : wm;   // omega_lambda
  R wml = lam > 0 ? wm : wp;  // omega_{-lambda}
  R s = R(double(lam));
  C4<R> v;
  v.c[0] = scale(c[0], -s * wl);
  v.c[1] = scale(c[1], -s * wl);
  v.c[2] = scale(c[0], s * wml);
  v.c[3] = scale(c[1], s * wml);
  return v;
}
// Massless vector boson polarisation, helicity lambda = +-1:
// eps = (-lambda e1 - i e2)/sqrt2, e1 = (0, cos t cos f, cos t sin f, -sin t),
// e2 = (0, -sin f, cos f, 0).  For an outgoing boson the conjugate is used.
template <class R> inline C4<R> polvec(const P4<R>& k, int lam, bool outgoing) {
  R kt = sqrt(k.x * k.x + k.y * k.y);
  R kk = sqrt(k.x * k.x + k.y * k.y + k.z * k.z);
  R ct = k.z / kk, st = kt / kk;
  R cf = R(1.0), sf = R(0.0);
  if (val(kt) > 0.0) { cf = k.x / kt; sf = k.y / kt; }
  R l = R(double(lam));
  R r2 = R(1.0 / std::sqrt(2.0));
  C4<R> e;
  e.c[0] = Cx<R>();
  e.c[1] = Cx<R>(-l * ct * cf * r2, sf * r2);
  e.c[2] = Cx<R>(-l * ct * sf * r2, -cf * r2);
  e.c[3] = Cx<R>(l * st * r2, R(0.0));
  if (outgoing)
    for (int i = 0; i < 4; ++i) e.c[i] = conj(e.c[i]);
  return e;
}

// ------------------------------------------------ colour-ordered recursion
// Colour-ordered Berends-Giele currents for a massive quark line t ... t~ with
// m gluons attached (all momenta outgoing), coupling set to 1:
//   J(s)   = [ -sum_splits V3(J_L, J_R) + sum_splits3 W4(J_A, J_B, J_C) ] / P_s^2
//   Psi(s) = -(pslash + m) [ sum_j slash(J(s_1..s_j)) Psi(s_{j+1}..) ] / (p^2 - m^2),
//            p = -p_tbar - P_s, Psi() = v(p_tbar)
//   A(s)   = sum_j ubar(p_t) slash(J(s_1..s_j)) Psi(s_{j+1}..s_m)
// with V3(X,Y) = X (2P_X+P_Y).Y + (X.Y)(P_Y-P_X) - Y (P_X+2P_Y).X and
// W4(A,B,C) = 2B(A.C) - A(B.C) - C(A.B).
template <class R> struct Recursion {
  int m;
  const C4<R>* eps;   // gluon external currents
  const P4<R>* k;     // gluon outgoing momenta
  C4<R> ubar, v;
  P4<R> ptb;          // antitop momentum
  R mt;
  std::vector<char> hj, hp;
  std::vector<C4<R>> mj, mp;
  static int code(const int* s, int n) {
    int c = 0;
    for (int i = 0; i < n; ++i) c = c * 7 + (s[i] + 1);
    return c;
  }
  void reset(int mm) {
    m = mm;
    int sz = 1;
    for (int i = 0; i < m; ++i) sz *= 7;
    hj.assign(sz, 0);
    hp.assign(sz, 0);
    mj.resize(sz);
    mp.resize(sz);
  }
  P4<R> mom(const int* s, int n) const {
    P4<R> P{R(0.0), R(0.0), R(0.0), R(0.0)};
    for (int i = 0; i < n; ++i) {
      P.e = P.e + k[s[i]].e;
      P.x = P.x + k[s[i]].x;
      P.y = P.y + k[s[i]].y;
      P.z = P.z + k[s[i]].z;
    }
    return P;
  }
  C4<R> J(const int* s, int n) {
    if (n == 1) return eps[s[0]];
    int c = code(s, n);
    if (hj[c]) return mj[c];
    C4<R> acc = c4zero<R>();
    for (int j = 1; j < n; ++j) {
      C4<R> X = J(s, j), Y = J(s + j, n - j);
      P4<R> PX = mom(s, j), PY = mom(s + j, n - j);
      P4<R> a{R(2.0) * PX.e + PY.e, R(2.0) * PX.x + PY.x, R(2.0) * PX.y + PY.y, R(2.0) * PX.z + PY.z};
      P4<R> b{PY.e - PX.e, PY.x - PX.x, PY.y - PX.y, PY.z - PX.z};
      P4<R> d{PX.e + R(2.0) * PY.e, PX.x + R(2.0) * PY.x, PX.y + R(2.0) * PY.y, PX.z + R(2.0) * PY.z};
      Cx<R> aY = cdot(fromP4(a), Y), XY = cdot(X, Y), dX = cdot(fromP4(d), X);
      C4<R> bb = fromP4(b);
      for (int mu = 0; mu < 4; ++mu)
        acc.c[mu] = acc.c[mu] - (X.c[mu] * aY + bb.c[mu] * XY - Y.c[mu] * dX);
    }
    for (int j = 1; j < n - 1; ++j)
      for (int l = j + 1; l < n; ++l) {
        C4<R> A = J(s, j), B = J(s + j, l - j), C = J(s + l, n - l);
        Cx<R> AC = cdot(A, C), BC = cdot(B, C), AB = cdot(A, B);
        for (int mu = 0; mu < 4; ++mu)
          acc.c[mu] = acc.c[mu] + (Cx<R>(R(2.0)) * B.c[mu] * AC - A.c[mu] * BC - C.c[mu] * AB);
      }
    P4<R> P = mom(s, n);
    R inv = R(1.0) / mdot(P, P);
    for (int mu = 0; mu < 4; ++mu) acc.c[mu] = scale(acc.c[mu], inv);
    hj[c] = 1;
    mj[c] = acc;
    return acc;
  }
  C4<R> Psi(const int* s, int n) {
    if (n == 0) return v;
    int c = code(s, n);
    if (hp[c]) return mp[c];
    C4<R> acc = c4zero<R>();
    for (int j = 1; j <= n; ++j) acc = c4add(acc, matvec(slash(J(s, j)), Psi(s + j, n - j)));
    P4<R> P = mom(s, n);
    P4<R> p{-ptb.e - P.e, -ptb.x - P.x, -ptb.y - P.y, -ptb.z - P.z};
    M4<R> ps = slash(fromP4(p));
    for (int i = 0; i < 4; ++i) ps.a[i][i] = ps.a[i][i] + Cx<R>(mt);
    R den = mdot(p, p) - mt * mt;
    C4<R> r = matvec(ps, acc);
    R f = R(-1.0) / den;
    for (int i = 0; i < 4; ++i) r.c[i] = scale(r.c[i], f);
    hp[c] = 1;
    mp[c] = r;
    return r;
  }
  Cx<R> amp(const int* s) {
    Cx<R> a;
    for (int j = 1; j <= m; ++j) a = a + rowvec(rowmat(ubar, slash(J(s, j))), Psi(s + j, m - j));
    return a;
  }
};

// Colour matrices C[sigma][sigma'] for m = 2..5 gluons on the quark line,
// orderings in lexicographic order; supplied by the caller (computed from
// explicit Gell-Mann matrices).
static std::vector<double> g_colour[6];

static void permutations(int m, std::vector<std::vector<int>>& out) {
  std::vector<int> p(m);
  for (int i = 0; i < m; ++i) p[i] = i;
  out.clear();
  do out.push_back(p);
  while (std::next_permutation(p.begin(), p.end()));
}

// Colour- and helicity-summed |M|^2 (coupling g = 1) for all-outgoing gluon
// momenta k[0..m-1] with given incoming/outgoing flags, top p_t, antitop p_tb.
// Optionally returns per-helicity values (2^(m+2) entries, gluon helicities
// in the high bits in gluon order, then top, then antitop; bit=1 -> +1).
template <class R>
R me_gluons(int m, const P4<R>* kphys, const bool* incoming, const P4<R>& pt, const P4<R>& ptb, R mt,
            double* per_hel) {
  const std::vector<double>& C = g_colour[m];
  std::vector<std::vector<int>> perms;
  permutations(m, perms);
  const int nf = (int)perms.size();
  std::vector<P4<R>> kout(m);
  for (int i = 0; i < m; ++i) {
    if (incoming[i]) kout[i] = P4<R>{-kphys[i].e, -kphys[i].x, -kphys[i].y, -kphys[i].z};
    else kout[i] = kphys[i];
  }
  std::vector<C4<R>> eps(m);
  std::vector<Cx<R>> A(nf);
  Recursion<R> rec;
  rec.k = kout.data();
  rec.eps = eps.data();
  rec.ptb = ptb;
  rec.mt = mt;
  R total = R(0.0);
  const int nhel = 1 << (m + 2);
  for (int h = 0; h < nhel; ++h) {
    for (int i = 0; i < m; ++i) {
      int lam = ((h >> (m + 1 - i)) & 1) ? 1 : -1;
      eps[i] = polvec(kphys[i], lam, !incoming[i]);
    }
    int lt = ((h >> 1) & 1) ? 1 : -1;
    int ltb = (h & 1) ? 1 : -1;
    rec.ubar = dbar(uspinor(pt, mt, lt));
    rec.v = vspinor(ptb, mt, ltb);
    rec.reset(m);
    for (int s = 0; s < nf; ++s) A[s] = rec.amp(perms[s].data());
    R mh = R(0.0);
    for (int s = 0; s < nf; ++s)
      for (int t = 0; t < nf; ++t) {
        Cx<R> z = conj(A[s]) * A[t];
        mh = mh + R(C[s * nf + t]) * z.re;
      }
    if (per_hel) per_hel[h] = val(mh);
    total = total + mh;
  }
  return total;
}

// q(p1) q~(p2) -> t(p3) t~(p4): one s-channel gluon. Colour sum
// sum_{a,b} Tr(t^a t^b)^2 = 2.  Returns colour- and helicity-summed |M|^2, g = 1.
template <class R>
R me_qqbar(const P4<R>& p1, const P4<R>& p2, const P4<R>& p3, const P4<R>& p4, R mt) {
  R zero(0.0);
  P4<R> s{p1.e + p2.e, p1.x + p2.x, p1.y + p2.y, p1.z + p2.z};
  R sh = mdot(s, s);
  R total = R(0.0);
  for (int h = 0; h < 16; ++h) {
    int l1 = (h & 8) ? 1 : -1, l2 = (h & 4) ? 1 : -1, l3 = (h & 2) ? 1 : -1, l4 = (h & 1) ? 1 : -1;
    C4<R> u1 = uspinor(p1, zero, l1);
    C4<R> vb2 = dbar(vspinor(p2, zero, l2));
    C4<R> ub3 = dbar(uspinor(p3, mt, l3));
    C4<R> v4 = vspinor(p4, mt, l4);
    // currents j^mu = psibar gamma^mu psi
    C4<R> jin, jout;
    for (int mu = 0; mu < 4; ++mu) {
      C4<R> e = c4zero<R>();
      e.c[mu] = Cx<R>(R(METRIC[mu]));  // slash(e) = gamma^mu with lowered index handled below
      M4<R> g = slash(e);              // = g_{mu mu} * METRIC[mu] gamma^mu = gamma^mu
      jin.c[mu] = rowvec(rowmat(vb2, g), u1);
      jout.c[mu] = rowvec(rowmat(ub3, g), v4);
    }
    Cx<R> a = cdot(jout, jin);
    R r = (a.re * a.re + a.im * a.im) / (sh * sh);
    total = total + r;
  }
  return R(2.0) * total;
}

// ------------------------------------------- two quark lines and one gluon
// Tree-level |M|^2 of q(p1) q~(p2) -> t(p3) t~(p4) g(p5) and of
// q(p1) g(p2) -> t(p3) t~(p4) q(p5), written diagram by diagram from the
// QCD Feynman rules in Feynman gauge: quark-gluon vertex i g gamma^mu t^a,
// fermion propagator i (pslash + m)/(p^2 - m^2), gluon propagator
// -i g_{mu nu} delta^{ab} / k^2, three-gluon vertex
// g f^{abc} [g^{mu nu}(k - p)^rho + g^{nu rho}(p - q)^mu + g^{rho mu}(q - k)^nu]
// for (a, mu, k), (b, nu, p), (c, rho, q) with all momenta incoming;
// coupling g = 1, light quarks massless.  Each process has five diagrams d
// with a Lorentz part K_d (its factors of i included) and a colour tensor
// C_d over (light-line colours, top-line colours, adjoint index of the
// external gluon):
//   d = 0: (t^b t^a)_{L}(t^b)_{T}   d = 1: (t^a t^b)_{L}(t^b)_{T}
//   d = 2: (t^c)_{L}(t^a t^c)_{T}   d = 3: (t^c)_{L}(t^c t^a)_{T}
//   d = 4: f^{abc}(t^b)_{L}(t^c)_{T}
// with L the light line (row index: the antiquark or the outgoing quark,
// column index: the incoming quark) and T the top line (row: top, column:
// antitop).  The colour- and helicity-summed |M|^2 is
//   sum_h sum_{d,d'} K_d K_d'^* CC[d][d'],  CC[d][d'] = sum_colours C_d C_d'^*,
// with CC supplied by the caller (explicit Gell-Mann matrices).
static std::vector<double> g_cc_re, g_cc_im;  // [5][5]

// J^mu = row gamma^mu col (contravariant components)
template <class R> inline C4<R> vec_current(const C4<R>& row, const C4<R>& col) {
  C4<R> J;
  for (int mu = 0; mu < 4; ++mu) {
    C4<R> e = c4zero<R>();
    e.c[mu] = Cx<R>(R(METRIC[mu]));  // slash(e) = gamma^mu
    J.c[mu] = rowvec(rowmat(row, slash(e)), col);
  }
  return J;
}
template <class R> inline P4<R> padd(const P4<R>& a, const P4<R>& b) { return P4<R>{a.e + b.e, a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class R> inline P4<R> psub(const P4<R>& a, const P4<R>& b) { return P4<R>{a.e - b.e, a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class R> inline P4<R> pneg(const P4<R>& a) { return P4<R>{-a.e, -a.x, -a.y, -a.z}; }
// (pslash + m) as a matrix
template <class R> inline M4<R> pslash_m(const P4<R>& p, R m) {
  M4<R> s = slash(fromP4(p));
  for (int i = 0; i < 4; ++i) s.a[i][i] = s.a[i][i] + Cx<R>(m);
  return s;
}
// three-gluon vertex contracted with the polarisations/currents of its legs:
// (a, rho, k, ea), (b, nu, p, eb), (c, mu, q, ec), all momenta incoming
template <class R>
inline Cx<R> v3g(const C4<R>& ea, const P4<R>& k, const C4<R>& eb, const P4<R>& p, const C4<R>& ec, const P4<R>& q) {
  return cdot(ea, eb) * cdot(fromP4(psub(k, p)), ec) + cdot(eb, ec) * cdot(fromP4(psub(p, q)), ea) +
         cdot(ec, ea) * cdot(fromP4(psub(q, k)), eb);
}

template <class R> inline R colour_contract(const Cx<R>* K) {
  R t = R(0.0);
  for (int d = 0; d < 5; ++d)
    for (int e = 0; e < 5; ++e) {
      Cx<R> z = K[d] * conj(K[e]);  // K_d K_e^*
      t = t + z.re * R(g_cc_re[5 * d + e]) - z.im * R(g_cc_im[5 * d + e]);
    }
  return t;
}

// q(p1) q~(p2) -> t(p3) t~(p4) g(p5): colour- and helicity-summed |M|^2, g = 1.
// ward = true replaces the gluon's polarisation by its momentum (the
// amplitude must then vanish for every colour).
template <class R>
R me_qqbar_g(const P4<R>& p1, const P4<R>& p2, const P4<R>& p3, const P4<R>& p4, const P4<R>& p5, R mt,
             bool ward = false) {
  const R zero(0.0);
  const P4<R> q12 = padd(p1, p2), q34 = padd(p3, p4);
  const R s12 = mdot(q12, q12), s34 = mdot(q34, q34);
  const P4<R> a1 = psub(p1, p5), a2 = psub(p5, p2), a3 = padd(p3, p5), a4 = pneg(padd(p4, p5));
  const R d1 = mdot(a1, a1), d2 = mdot(a2, a2), d3 = mdot(a3, a3) - mt * mt, d4 = mdot(a4, a4) - mt * mt;
  const Cx<R> mi(R(0.0), R(-1.0));  // -i of the diagrams with two fermion propagators' worth of i
  R total = R(0.0);
  for (int h = 0; h < 32; ++h) {
    const int l1 = (h & 16) ? 1 : -1, l2 = (h & 8) ? 1 : -1, l3 = (h & 4) ? 1 : -1, l4 = (h & 2) ? 1 : -1,
              l5 = (h & 1) ? 1 : -1;
    const C4<R> u1 = uspinor(p1, zero, l1);
    const C4<R> vb2 = dbar(vspinor(p2, zero, l2));
    const C4<R> ub3 = dbar(uspinor(p3, mt, l3));
    const C4<R> v4 = vspinor(p4, mt, l4);
    const C4<R> e5 = ward ? fromP4(p5) : polvec(p5, l5, true);  // eps* of the outgoing gluon
    const M4<R> E5 = slash(e5);
    const C4<R> J12 = vec_current(vb2, u1), J34 = vec_current(ub3, v4);
    Cx<R> K[5];
    // d0: emission from the incoming quark
    {
      const C4<R> L = vec_current(vb2, matvec(slash(fromP4(a1)), matvec(E5, u1)));
      K[0] = mi * scale(cdot(L, J34), R(1.0) / (d1 * s34));
    }
    // d1: emission from the incoming antiquark
    {
      const C4<R> L = vec_current(rowmat(rowmat(vb2, E5), slash(fromP4(a2))), u1);
      K[1] = mi * scale(cdot(L, J34), R(1.0) / (d2 * s34));
    }
    // d2: emission from the top
    {
      const C4<R> T = vec_current(rowmat(rowmat(ub3, E5), pslash_m(a3, mt)), v4);
      K[2] = mi * scale(cdot(T, J12), R(1.0) / (d3 * s12));
    }
    // d3: emission from the antitop
    {
      const C4<R> T = vec_current(ub3, matvec(pslash_m(a4, mt), matvec(E5, v4)));
      K[3] = mi * scale(cdot(T, J12), R(1.0) / (d4 * s12));
    }
    // d4: three-gluon vertex: (a, -p5, e5), (b, p1 + p2, J12), (c, -(p3 + p4), J34)
    K[4] = scale(v3g(e5, pneg(p5), J12, q12, J34, pneg(q34)), R(1.0) / (s12 * s34));
    total = total + colour_contract(K);
  }
  return total;
}

// q(p1) g(p2) -> t(p3) t~(p4) q(p5): colour- and helicity-summed |M|^2, g = 1.
template <class R>
R me_qg_q(const P4<R>& p1, const P4<R>& p2, const P4<R>& p3, const P4<R>& p4, const P4<R>& p5, R mt,
          bool ward = false) {
  const R zero(0.0);
  const P4<R> q12 = padd(p1, p2), q34 = padd(p3, p4), q15 = psub(p1, p5);
  const R s12 = mdot(q12, q12), s34 = mdot(q34, q34), t15 = mdot(q15, q15);
  const P4<R> a2 = psub(p5, p2), a3 = psub(p3, p2), a4 = psub(p2, p4);
  const R d2 = mdot(a2, a2), d3 = mdot(a3, a3) - mt * mt, d4 = mdot(a4, a4) - mt * mt;
  const Cx<R> mi(R(0.0), R(-1.0));
  R total = R(0.0);
  for (int h = 0; h < 32; ++h) {
    const int l1 = (h & 16) ? 1 : -1, l2 = (h & 8) ? 1 : -1, l3 = (h & 4) ? 1 : -1, l4 = (h & 2) ? 1 : -1,
              l5 = (h & 1) ? 1 : -1;
    const C4<R> u1 = uspinor(p1, zero, l1);
    const C4<R> e2 = ward ? fromP4(p2) : polvec(p2, l2, false);  // eps of the incoming gluon
    const M4<R> E2 = slash(e2);
    const C4<R> ub3 = dbar(uspinor(p3, mt, l3));
    const C4<R> v4 = vspinor(p4, mt, l4);
    const C4<R> ub5 = dbar(uspinor(p5, zero, l5));
    const C4<R> J15 = vec_current(ub5, u1), J34 = vec_current(ub3, v4);
    Cx<R> K[5];
    // d0: s-channel quark (the gluon absorbed first)
    {
      const C4<R> L = vec_current(ub5, matvec(slash(fromP4(q12)), matvec(E2, u1)));
      K[0] = mi * scale(cdot(L, J34), R(1.0) / (s12 * s34));
    }
    // d1: u-channel quark (the gluon absorbed after the emission of the top pair)
    {
      const C4<R> L = vec_current(rowmat(rowmat(ub5, E2), slash(fromP4(a2))), u1);
      K[1] = mi * scale(cdot(L, J34), R(1.0) / (d2 * s34));
    }
    // d2: t-channel gluon, the incoming gluon attached next to the top
    {
      const C4<R> T = vec_current(rowmat(rowmat(ub3, E2), pslash_m(a3, mt)), v4);
      K[2] = mi * scale(cdot(T, J15), R(1.0) / (d3 * t15));
    }
    // d3: t-channel gluon, the incoming gluon attached next to the antitop
    {
      const C4<R> T = vec_current(ub3, matvec(pslash_m(a4, mt), matvec(E2, v4)));
      K[3] = mi * scale(cdot(T, J15), R(1.0) / (d4 * t15));
    }
    // d4: three-gluon vertex: (a, p2, e2), (b, p1 - p5, J15), (c, -(p3 + p4), J34)
    K[4] = scale(v3g(e2, p2, J15, q15, J34, pneg(q34)), R(1.0) / (t15 * s34));
    total = total + colour_contract(K);
  }
  return total;
}

// ----------------------------------------------------------------- Philox
static inline void mulhilo(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  hi = (uint64_t)(p >> 64);
  lo = (uint64_t)p;
}
// Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).
static void philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo(M0, x0, hi0, lo0);
    mulhilo(M1, x2, hi1, lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}
static inline double u01(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1.0p-53; }

// The uniforms of one event: counter (event, iteration, call, 0), key (seed, purpose).
static void event_uniforms(uint64_t ev, uint64_t it, uint64_t seed, uint64_t purpose, int d, double* u) {
  uint64_t key[2] = {seed, purpose};
  for (int call = 0; call * 4 < d; ++call) {
    uint64_t ctr[4] = {ev, it, (uint64_t)call, 0};
    uint64_t o[4];
    philox4x64_10(ctr, key, o);
    for (int w = 0; w < 4 && call * 4 + w < d; ++w) u[call * 4 + w] = u01(o[w]);
  }
}

// ---------------------------------------------------------------- VEGAS
// y in (0,1)^d -> x through the piecewise-linear map of adaptive bins.
static double vegas_map(const double* edges, int d, int nb, const double* y, double* x, int* bins) {
  double jac = 1.0;
  for (int j = 0; j < d; ++j) {
    double t = y[j] * nb;
    int k = (int)std::floor(t);
    if (k >= nb) k = nb - 1;
    if (k < 0) k = 0;
    const double* e = edges + (size_t)j * (nb + 1);
    double w = e[k + 1] - e[k];
    x[j] = e[k] + (t - k) * w;
    jac *= nb * w;
    bins[j] = k;
  }
  return jac;
}

// Lepage's refinement of one dimension: 3-point smoothing of the bin sums,
// damped importance r_k = [(1 - d_k/D)/ln(D/d_k)]^alpha, then new edges
// carrying equal shares of sum r, linearly interpolated inside old bins.
static void refine_dim(double* e, const double* hist, int nb, double alpha) {
  std::vector<double> d(nb), r(nb);
  if (nb == 1) { d[0] = hist[0]; }
  else {
    d[0] = 0.5 * (hist[0] + hist[1]);
    d[nb - 1] = 0.5 * (hist[nb - 2] + hist[nb - 1]);
    for (int k = 1; k < nb - 1; ++k) d[k] = (hist[k - 1] + hist[k] + hist[k + 1]) / 3.0;
  }
  double D = 0.0;
  for (int k = 0; k < nb; ++k) D += d[k];
  if (!(D > 0.0)) return;
  double R = 0.0;
  for (int k = 0; k < nb; ++k) {
    if (d[k] > 0.0) {
      double q = d[k] / D;
      r[k] = (q < 1.0) ? std::pow((1.0 - q) / std::log(1.0 / q), alpha) : 0.0;
    } else r[k] = 0.0;
    R += r[k];
  }
  if (!(R > 0.0)) return;
  std::vector<double> old(e, e + nb + 1), ne(nb + 1);
  double per = R / nb;
  ne[0] = old[0];
  ne[nb] = old[nb];
  // Walk through old bins, accumulating importance.
  int k = 0;
  double acc = 0.0;  // importance of old bins fully consumed before bin k
  for (int i = 1; i < nb; ++i) {
    double target = per * i;
    while (k < nb && acc + r[k] < target) {
      acc += r[k];
      ++k;
    }
    if (k >= nb) { ne[i] = old[nb]; continue; }
    double frac = (target - acc) / r[k];
    ne[i] = old[k] + frac * (old[k + 1] - old[k]);
  }
  for (int i = 0; i <= nb; ++i) e[i] = ne[i];
}

// ----------------------------------------------------------------- PDFs
// Synthetic x f(x,Q) = A x^(a + b L) (1-x)^(c + d L), L = ln(Q / 1.65 GeV),
// tabulated at x_i = 10^(-9 + 9 i/195), i = 0..195 and
// Q_j = 1.65 (1e5/1.65)^(j/49), j = 0..49, for flavours g, u, d, u~.
static const int NX = 196, NQ = 50;
static const double Q0 = 1.65, QMAX = 1e5;
static inline double xknot(int i) { return std::pow(10.0, -9.0 + 9.0 * i / 195.0); }
static inline double qknot(int j) { return Q0 * std::pow(QMAX / Q0, j / 49.0); }

// Analytic value and parameter derivatives (index 0..4 = A,a,b,c,d) at (x,Q).
static double pdf_formula(const double* p5, double x, double Q, int dpar) {
  double L = std::log(Q / Q0);
  if (x >= 1.0) return 0.0;
  double lx = std::log(x), l1x = std::log1p(-x);
  double v = p5[0] * std::exp((p5[1] + p5[2] * L) * lx + (p5[3] + p5[4] * L) * l1x);
  switch (dpar) {
    case -1: return v;
    case 0: return v / p5[0];
    case 1: return v * lx;
    case 2: return v * L * lx;
    case 3: return v * l1x;
    case 4: return v * L * l1x;
  }
  return 0.0;
}

// One-dimensional cubic Hermite on unit-spaced knots f[0..n-1] with
// central-difference slopes (one-sided at the two end knots), at fractional
// position t in [0, n-1].
template <class R> static R hermite1(const R* f, int n, R t) {
  int i = (int)std::floor(val(t));
  if (i < 0) i = 0;
  if (i > n - 2) i = n - 2;
  R u = t - R(double(i));
  R s0 = (i == 0) ? f[1] - f[0] : (f[i + 1] - f[i - 1]) * R(0.5);
  R s1 = (i + 1 == n - 1) ? f[n - 1] - f[n - 2] : (f[i + 2] - f[i]) * R(0.5);
  R u2 = u * u, u3 = u2 * u;
  R h00 = R(2.0) * u3 - R(3.0) * u2 + R(1.0);
  R h10 = u3 - R(2.0) * u2 + u;
  R h01 = R(-2.0) * u3 + R(3.0) * u2;
  R h11 = u3 - u2;
  return h00 * f[i] + h10 * s0 + h01 * f[i + 1] + h11 * s1;
}

// Tensor-product Hermite: interpolate in ln x along every Q row, then in ln Q.
// table[j*NX + i]; returns x f(x, Q).
template <class R> static R pdf_interp(const R* table, double x, R Q) {
  double tx = (std::log(x) - std::log(xknot(0))) / ((std::log(xknot(NX - 1)) - std::log(xknot(0))) / (NX - 1));
  R tq = (log(Q) - R(std::log(Q0))) / R((std::log(QMAX) - std::log(Q0)) / (NQ - 1));
  std::vector<R> col(NQ);
  for (int j = 0; j < NQ; ++j) col[j] = hermite1(table + (size_t)j * NX, NX, R(tx));
  return hermite1(col.data(), NQ, tq);
}

// ---------------------------------------------------------- configuration
extern "C" {
typedef struct {
  int n_g;       // final-state gluons for the gluon channel (0..3)
  int channel;   // 0: g g, 1: u u~ (+ u~ u), 2: d d~ (+ d~ d)
  double sqrt_s, m_t, mu, alpha_s, pt_min, eta_max, dr_min;
  double pdf[20];  // (A,a,b,c,d) for g, u, d, u~
  int dyn_scale;   // 1: factorisation scale mu = H_T / 2 per event (else mu / m_t)
} or_cfg;
}

// Per-configuration state: PDF tables (values and one derivative table per
// gradient direction).
struct State {
  or_cfg cfg;
  std::vector<double> tab[4];       // values per flavour
  std::vector<double> dtab[4][5];   // d(xf)/d(param) per flavour and parameter
};

static void build_tables(State& S) {
  for (int f = 0; f < 4; ++f) {
    S.tab[f].assign((size_t)NX * NQ, 0.0);
    for (int p = 0; p < 5; ++p) S.dtab[f][p].assign((size_t)NX * NQ, 0.0);
    for (int j = 0; j < NQ; ++j)
      for (int i = 0; i < NX; ++i) {
        double x = xknot(i), Q = qknot(j);
        S.tab[f][(size_t)j * NX + i] = pdf_formula(S.cfg.pdf + 5 * f, x, Q, -1);
        for (int p = 0; p < 5; ++p) S.dtab[f][p][(size_t)j * NX + i] = pdf_formula(S.cfg.pdf + 5 * f, x, Q, p);
      }
  }
}

// Gradient direction: 0 none, 1 m_t, 2..9 theta = (A_g, a_g, b_g, c_g, d_g, A_u, A_d, A_u~).
static void theta_index(int dir, int& flav, int& par) {
  flav = -1; par = -1;
  if (dir >= 2 && dir <= 6) { flav = 0; par = dir - 2; }
  else if (dir == 7) { flav = 1; par = 0; }
  else if (dir == 8) { flav = 2; par = 0; }
  else if (dir == 9) { flav = 3; par = 0; }
}

// PDF value of flavour f at (x, mu) as a dual in direction dir.
static Dual pdf_dual(const State& S, int f, double x, Dual mu, int dir) {
  int fl, par;
  theta_index(dir, fl, par);
  std::vector<Dual> t((size_t)NX * NQ);
  for (size_t i = 0; i < t.size(); ++i)
    t[i] = Dual(S.tab[f][i], (fl == f) ? S.dtab[f][par][i] : 0.0);
  return pdf_interp(t.data(), x, mu);
}
static double pdf_val(const State& S, int f, double x, double mu) { return pdf_interp(S.tab[f].data(), x, mu); }

// ------------------------------------------------------------ phase space
template <class R> static P4<R> boost_from_rest(const P4<R>& p, const P4<R>& Q, R M) {
  // p given in the rest frame of Q; returns p in the frame where Q has momentum Q.
  R bp = Q.x * p.x + Q.y * p.y + Q.z * p.z;
  R e = (Q.e * p.e + bp) / M;
  R c = (bp / (Q.e + M) + p.e) / M;
  return P4<R>{e, p.x + c * Q.x, p.y + c * Q.y, p.z + c * Q.z};
}

// Solve (N-1) v^(N-2) - (N-2) v^(N-1) = r for v in [0,1] by bisection
// (the CDF of v = M_i^2 / M_{i-1}^2 for N massless particles).
static double solve_mass_ratio(int N, double r) {
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    double F = (N - 1) * std::pow(mid, N - 2) - (N - 2) * std::pow(mid, N - 1);
    if (F < r) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

static double factorial(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

// Massless n-body phase-space volume V_n(s) including (2 pi)^(4-3n).
static double massless_volume(int n, double s) {
  return std::pow(2.0 * M_PI, 4.0 - 3.0 * n) * std::pow(M_PI / 2.0, n - 1) * std::pow(s, n - 2) /
         (factorial(n - 1) * factorial(n - 2));
}

// Build the final state in the partonic CM frame from uniforms x[2..].
// Outputs: out[0..ng-1] gluons (emission order), out[ng] top, out[ng+1] antitop.
// Returns the weight V_n * beta, or 0 below the t t~ threshold.
template <class R>
static R phase_space(int ng, const double* x, double shat, R mt, P4<R>* out) {
  const int n = ng + 2;
  double M = std::sqrt(shat);
  P4<R> Q{R(M), R(0.0), R(0.0), R(0.0)};
  double Mprev = M;
  for (int i = 1; i <= n - 2; ++i) {
    double r = x[2 + (i - 1)];
    int N = n - i + 1;  // particles in the system being split
    double v = solve_mass_ratio(N, r);
    double Mi = Mprev * std::sqrt(v);
    double q = (Mprev * Mprev - Mi * Mi) / (2.0 * Mprev);
    double ct = 2.0 * x[2 + (n - 2) + 2 * (i - 1)] - 1.0;
    double phi = 2.0 * M_PI * x[2 + (n - 2) + 2 * (i - 1) + 1];
    double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
    P4<R> g{R(q), R(q * st * std::cos(phi)), R(q * st * std::sin(phi)), R(q * ct)};
    P4<R> rest{R(std::sqrt(Mi * Mi + q * q)), -g.x, -g.y, -g.z};
    out[i - 1] = boost_from_rest(g, Q, R(Mprev));
    Q = boost_from_rest(rest, Q, R(Mprev));
    Mprev = Mi;
  }
  R Mtt = R(Mprev);
  if (!(val(Mtt) > 2.0 * val(mt))) return R(0.0);
  R beta = sqrt(R(1.0) - R(4.0) * mt * mt / (Mtt * Mtt));
  R q = Mtt * beta * R(0.5);
  double ct = 2.0 * x[2 + (n - 2) + 2 * (n - 2)] - 1.0;
  double phi = 2.0 * M_PI * x[2 + (n - 2) + 2 * (n - 2) + 1];
  double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
  R E = Mtt * R(0.5);
  P4<R> t{E, q * R(st * std::cos(phi)), q * R(st * std::sin(phi)), q * R(ct)};
  P4<R> tb{E, -t.x, -t.y, -t.z};
  out[ng] = boost_from_rest(t, Q, Mtt);
  out[ng + 1] = boost_from_rest(tb, Q, Mtt);
  return R(massless_volume(n, shat)) * beta;
}

// Fiducial cuts on the gluons, evaluated in the lab frame (longitudinal boost
// by rapidity y = ln(x1/x2)/2): pT > ptmin, |eta| < etamax, pairwise dR > drmin.
static bool pass_cuts(const or_cfg& c, int ng, const P4<double>* g, double x1, double x2) {
  if (ng == 0) return true;
  double y = 0.5 * std::log(x1 / x2);
  double ch = std::cosh(y), sh = std::sinh(y);
  std::vector<double> eta(ng), phi(ng);
  for (int i = 0; i < ng; ++i) {
    double pt = std::sqrt(g[i].x * g[i].x + g[i].y * g[i].y);
    double pz = g[i].z * ch + g[i].e * sh;
    double pp = std::sqrt(pt * pt + pz * pz);
    if (!(pt > c.pt_min)) return false;
    eta[i] = std::atanh(pz / pp);
    if (!(std::fabs(eta[i]) < c.eta_max)) return false;
    phi[i] = std::atan2(g[i].y, g[i].x);
  }
  if (c.dr_min > 0.0)
    for (int i = 0; i < ng; ++i)
      for (int j = i + 1; j < ng; ++j) {
        double dphi = phi[i] - phi[j];
        while (dphi > M_PI) dphi -= 2.0 * M_PI;
        while (dphi < -M_PI) dphi += 2.0 * M_PI;
        double de = eta[i] - eta[j];
        if (!(std::sqrt(de * de + dphi * dphi) > c.dr_min)) return false;
      }
  return true;
}

static const double GEV2_TO_PB = 3.893793721e8;

// The integrand w(x) in pb for x in the unit hypercube (after the VEGAS map),
// as a dual number in direction dir.  Also returns the momenta if asked.
template <class R>
static R integrand_T(const State& S, const double* x, R mt, int dir, double* mom_out, int* pass_out) {
  const or_cfg& c = S.cfg;
  // gluons (g g channel) or one light parton (quark channels with n_g = 1)
  const int ng = c.n_g;
  const int n = ng + 2;
  if (pass_out) *pass_out = 0;
  double s = c.sqrt_s * c.sqrt_s;
  double x1 = x[0], x2 = x[1];
  double shat = x1 * x2 * s;
  if (!(shat > 4.0 * val(mt) * val(mt))) return R(0.0);
  std::vector<P4<R>> fs(n);
  R wps = phase_space<R>(ng, x, shat, mt, fs.data());
  if (val(wps) == 0.0) return R(0.0);
  std::vector<P4<double>> gl(ng);
  for (int i = 0; i < ng; ++i) gl[i] = P4<double>{val(fs[i].e), val(fs[i].x), val(fs[i].y), val(fs[i].z)};
  if (mom_out) {
    double E = 0.5 * std::sqrt(shat);
    double* o = mom_out;
    double in[8] = {E, 0, 0, E, E, 0, 0, -E};
    for (int i = 0; i < 8; ++i) o[i] = in[i];
    // order: p1, p2, top, antitop, gluons
    const P4<R>* ord[8];
    ord[0] = &fs[ng];
    ord[1] = &fs[ng + 1];
    for (int i = 0; i < ng; ++i) ord[2 + i] = &fs[i];
    for (int i = 0; i < n; ++i) {
      o[8 + 4 * i + 0] = val(ord[i]->e);
      o[8 + 4 * i + 1] = val(ord[i]->x);
      o[8 + 4 * i + 2] = val(ord[i]->y);
      o[8 + 4 * i + 3] = val(ord[i]->z);
    }
  }
  if (!pass_cuts(c, ng, gl.data(), x1, x2)) return R(0.0);
  if (pass_out) *pass_out = 1;
  R mu = (c.mu > 0.0) ? R(c.mu) : mt;
  if (c.dyn_scale) {
    // mu = H_T / 2: half the sum of the transverse masses of the final state
    // (the tops with mass m_t, the massless gluons)
    const P4<R>& t = fs[ng];
    const P4<R>& tb = fs[ng + 1];
    R ht = sqrt(mt * mt + t.x * t.x + t.y * t.y) + sqrt(mt * mt + tb.x * tb.x + tb.y * tb.y);
    for (int i = 0; i < ng; ++i) ht = ht + sqrt(fs[i].x * fs[i].x + fs[i].y * fs[i].y);
    mu = ht * R(0.5);
  }
  double E = 0.5 * std::sqrt(shat);
  P4<R> p1{R(E), R(0.0), R(0.0), R(E)}, p2{R(E), R(0.0), R(0.0), R(-E)};
  double gs2 = 4.0 * M_PI * c.alpha_s;  // g^2
  R me;
  R lum;
  if (c.channel == 0) {
    const int m = ng + 2;
    std::vector<P4<R>> kph(m);
    std::vector<char> inc(m);
    kph[0] = p1; inc[0] = 1;
    kph[1] = p2; inc[1] = 1;
    for (int i = 0; i < ng; ++i) { kph[2 + i] = fs[i]; inc[2 + i] = 0; }
    bool incb[8];
    for (int i = 0; i < m; ++i) incb[i] = inc[i] != 0;
    R sum = me_gluons<R>(m, kph.data(), incb, fs[ng], fs[ng + 1], mt, nullptr);
    me = sum * R(std::pow(gs2, m) / 256.0 / factorial(ng));
    R f1, f2;
    if constexpr (std::is_same<R, Dual>::value) {
      f1 = pdf_dual(S, 0, x1, mu, dir);
      f2 = pdf_dual(S, 0, x2, mu, dir);
    } else {
      f1 = pdf_val(S, 0, x1, mu);
      f2 = pdf_val(S, 0, x2, mu);
    }
    lum = f1 * f2 / R(x1 * x2);
  } else if (ng == 1) {
    // quark channels with one more parton: the light parton is fs[0], the
    // top pair fs[1], fs[2]
    auto pdf = [&](int f, double x) -> R {
      if constexpr (std::is_same<R, Dual>::value) return pdf_dual(S, f, x, mu, dir);
      else return pdf_val(S, f, x, mu);
    };
    if (c.channel == 1 || c.channel == 2) {
      // q q~ -> t t~ g, the quark from either beam
      const int q = (c.channel == 1) ? 1 : 2;
      R m12 = me_qqbar_g<R>(p1, p2, fs[1], fs[2], fs[0], mt);
      R m21 = me_qqbar_g<R>(p2, p1, fs[1], fs[2], fs[0], mt);
      R sc = R(gs2 * gs2 * gs2 / 36.0 / (x1 * x2));
      me = R(1.0);
      lum = (pdf(q, x1) * pdf(3, x2) * m12 + pdf(3, x1) * pdf(q, x2) * m21) * sc;
    } else {
      // q g -> t t~ q for q = u, d from either beam, and q~ g -> t t~ q~ for
      // q~ = u~, d~ (equal PDFs): by charge conjugation |M(q~ g -> t t~ q~)|^2
      // is |M(q g -> t t~ q)|^2 with the top and antitop momenta exchanged
      R mq12 = me_qg_q<R>(p1, p2, fs[1], fs[2], fs[0], mt);
      R mq21 = me_qg_q<R>(p2, p1, fs[1], fs[2], fs[0], mt);
      R ma12 = me_qg_q<R>(p1, p2, fs[2], fs[1], fs[0], mt);
      R ma21 = me_qg_q<R>(p2, p1, fs[2], fs[1], fs[0], mt);
      R g1 = pdf(0, x1), g2 = pdf(0, x2);
      R qs1 = pdf(1, x1) + pdf(2, x1), qs2 = pdf(1, x2) + pdf(2, x2);
      R as1 = R(2.0) * pdf(3, x1), as2 = R(2.0) * pdf(3, x2);
      R sc = R(gs2 * gs2 * gs2 / 96.0 / (x1 * x2));
      me = R(1.0);
      lum = (qs1 * g2 * mq12 + g1 * qs2 * mq21 + as1 * g2 * ma12 + g1 * as2 * ma21) * sc;
    }
  } else {
    int q = (c.channel == 1) ? 1 : 2;
    R sum12 = me_qqbar<R>(p1, p2, fs[0], fs[1], mt);  // quark from beam 1
    R sum21 = me_qqbar<R>(p2, p1, fs[0], fs[1], mt);  // quark from beam 2
    R fq1, fq2, fa1, fa2;
    if constexpr (std::is_same<R, Dual>::value) {
      fq1 = pdf_dual(S, q, x1, mu, dir); fa2 = pdf_dual(S, 3, x2, mu, dir);
      fa1 = pdf_dual(S, 3, x1, mu, dir); fq2 = pdf_dual(S, q, x2, mu, dir);
    } else {
      fq1 = pdf_val(S, q, x1, mu); fa2 = pdf_val(S, 3, x2, mu);
      fa1 = pdf_val(S, 3, x1, mu); fq2 = pdf_val(S, q, x2, mu);
    }
    R sc = R(gs2 * gs2 / 36.0 / (x1 * x2));
    // |M|^2 for each beam assignment times its parton luminosity
    me = R(1.0);
    lum = (fq1 * fa2 * sum12 + fa1 * fq2 * sum21) * sc;
  }
  R w = lum * me * wps * R(GEV2_TO_PB / (2.0 * shat));
  return w;
}

static std::vector<State*> g_states;

}  // namespace orc

using namespace orc;

extern "C" {

int or_version(void) { return 1; }

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_philox4x64_10(const uint64_t* ctr, const uint64_t* key, uint64_t* out) { philox4x64_10(ctr, key, out); }

void or_event_uniforms(uint64_t n, uint64_t ev0, uint64_t it, uint64_t seed, uint64_t purpose, int d, double* u) {
  // u is [n][d] row-major
  for (uint64_t e = 0; e < n; ++e) event_uniforms(ev0 + e, it, seed, purpose, d, u + e * d);
}

double or_vegas_map(const double* edges, int d, int nb, const double* y, double* x, int* bins) {
  return vegas_map(edges, d, nb, y, x, bins);
}

void or_vegas_refine(double* edges, const double* hist, int d, int nb, double alpha) {
  for (int j = 0; j < d; ++j) refine_dim(edges + (size_t)j * (nb + 1), hist + (size_t)j * nb, nb, alpha);
}

void or_set_colour_qq(const double* re, const double* im) {
  g_cc_re.assign(re, re + 25);
  g_cc_im.assign(im, im + 25);
}

// The two-quark-line matrix elements at explicit physical momenta
// mom = (p1, p2, p3, p4, p5) [5][4]; kind 0: q q~ -> t t~ g, 1: q g -> t t~ q;
// ward = 1: the gluon's polarisation replaced by its momentum.
double or_me_qq(int kind, const double* mom, double mt, int ward) {
  P4<double> p[5];
  for (int i = 0; i < 5; ++i) p[i] = P4<double>{mom[4 * i], mom[4 * i + 1], mom[4 * i + 2], mom[4 * i + 3]};
  return kind == 0 ? me_qqbar_g<double>(p[0], p[1], p[2], p[3], p[4], mt, ward != 0)
                   : me_qg_q<double>(p[0], p[1], p[2], p[3], p[4], mt, ward != 0);
}

void or_set_colour(int m, int nf, const double* C) {
  if (m < 2 || m > 5) return;
  g_colour[m].assign(C, C + (size_t)nf * nf);
}

int or_state_create(const or_cfg* c) {
  State* S = new State();
  S->cfg = *c;
  build_tables(*S);
  g_states.push_back(S);
  return (int)g_states.size() - 1;
}

void or_state_destroy(int h) {
  if (h >= 0 && h < (int)g_states.size()) { delete g_states[h]; g_states[h] = nullptr; }
}

// The fiducial cut decision of a configured state for explicit partonic-frame
// gluon momenta g[ng][4] and momentum fractions x1, x2 (1 = every cut passed).
int or_pass_cuts(int h, int ng, const double* g, double x1, double x2) {
  std::vector<P4<double>> gl(ng);
  for (int i = 0; i < ng; ++i) gl[i] = P4<double>{g[4 * i], g[4 * i + 1], g[4 * i + 2], g[4 * i + 3]};
  return pass_cuts(g_states[h]->cfg, ng, gl.data(), x1, x2) ? 1 : 0;
}

void or_pdf_table(int h, int f, double* out) {
  const State& S = *g_states[h];
  std::copy(S.tab[f].begin(), S.tab[f].end(), out);
}

// x f(x,Q) by interpolation, or the analytic formula (analytic != 0).
void or_pdf(int h, int f, int n, const double* x, const double* Q, int analytic, double* out) {
  const State& S = *g_states[h];
  for (int i = 0; i < n; ++i)
    out[i] = analytic ? pdf_formula(S.cfg.pdf + 5 * f, x[i], Q[i], -1) : pdf_val(S, f, x[i], Q[i]);
}

// Interpolate an arbitrary user table (NQ x NX) -- used to test the interpolant
// on functions it must reproduce.
void or_hermite2d(const double* table, int n, const double* x, const double* Q, double* out) {
  for (int i = 0; i < n; ++i) out[i] = pdf_interp(table, x[i], Q[i]);
}

// Phase space: x is [n_events][d]; mom is [n_events][n_ext][4] in the order
// (p1, p2, top, antitop, gluons...); weight [n_events].
void or_phase_space(int ng, int nev, const double* x, double sqrt_shat, double mt, double* mom, double* wt) {
  const int n = ng + 2, d = 3 * n - 2;
  for (int e = 0; e < nev; ++e) {
    std::vector<P4<double>> fs(n);
    double shat = sqrt_shat * sqrt_shat;
    double w = phase_space<double>(ng, x + (size_t)e * d, shat, mt, fs.data());
    wt[e] = w;
    double E = 0.5 * sqrt_shat;
    double* o = mom + (size_t)e * 4 * (n + 2);
    double in[8] = {E, 0, 0, E, E, 0, 0, -E};
    for (int i = 0; i < 8; ++i) o[i] = in[i];
    const P4<double>* ord[8];
    ord[0] = &fs[ng];
    ord[1] = &fs[ng + 1];
    for (int i = 0; i < ng; ++i) ord[2 + i] = &fs[i];
    for (int i = 0; i < n; ++i) {
      o[8 + 4 * i + 0] = ord[i]->e;
      o[8 + 4 * i + 1] = ord[i]->x;
      o[8 + 4 * i + 2] = ord[i]->y;
      o[8 + 4 * i + 3] = ord[i]->z;
    }
  }
}

// Colour- and helicity-summed |M|^2 (g = 1) for g g -> t t~ + (m-2) g.
// mom: (p1, p2, top, antitop, gluons...) physical momenta, p1 and p2 incoming.
// per_hel (optional): 2^(m+2) values.
double or_me_gg(int m, const double* mom, double mt, double* per_hel) {
  std::vector<P4<double>> k(m);
  bool inc[8];
  k[0] = P4<double>{mom[0], mom[1], mom[2], mom[3]};
  k[1] = P4<double>{mom[4], mom[5], mom[6], mom[7]};
  inc[0] = inc[1] = true;
  for (int i = 2; i < m; ++i) {
    const double* p = mom + 16 + 4 * (i - 2);
    k[i] = P4<double>{p[0], p[1], p[2], p[3]};
    inc[i] = false;
  }
  P4<double> pt{mom[8], mom[9], mom[10], mom[11]}, ptb{mom[12], mom[13], mom[14], mom[15]};
  return me_gluons<double>(m, k.data(), inc, pt, ptb, mt, per_hel);
}

// Generic all-outgoing variant for invariance tests: gluon momenta k[m][4]
// with flags incoming[m] (1 = physical incoming momentum given), optional
// replacement of gluon `ward` polarisation by its momentum (-1 = none).
// Returns the partial amplitudes A[nf] (re, im interleaved) for helicity h.
void or_partial_amps(int m, const double* kin, const int* incoming, const double* pt, const double* ptb, double mt,
                     int h, int ward, double* amps) {
  std::vector<P4<double>> kph(m), kout(m);
  for (int i = 0; i < m; ++i) {
    kph[i] = P4<double>{kin[4 * i], kin[4 * i + 1], kin[4 * i + 2], kin[4 * i + 3]};
    kout[i] = incoming[i] ? P4<double>{-kph[i].e, -kph[i].x, -kph[i].y, -kph[i].z} : kph[i];
  }
  std::vector<C4<double>> eps(m);
  for (int i = 0; i < m; ++i) {
    int lam = ((h >> (m + 1 - i)) & 1) ? 1 : -1;
    eps[i] = polvec(kph[i], lam, !incoming[i]);
    if (i == ward) eps[i] = fromP4(kout[i]);
  }
  P4<double> Pt{pt[0], pt[1], pt[2], pt[3]}, Ptb{ptb[0], ptb[1], ptb[2], ptb[3]};
  int lt = ((h >> 1) & 1) ? 1 : -1, ltb = (h & 1) ? 1 : -1;
  Recursion<double> rec;
  rec.k = kout.data();
  rec.eps = eps.data();
  rec.ptb = Ptb;
  rec.mt = mt;
  rec.ubar = dbar(uspinor(Pt, mt, lt));
  rec.v = vspinor(Ptb, mt, ltb);
  rec.reset(m);
  std::vector<std::vector<int>> perms;
  permutations(m, perms);
  for (size_t s = 0; s < perms.size(); ++s) {
    Cx<double> a = rec.amp(perms[s].data());
    amps[2 * s] = a.re;
    amps[2 * s + 1] = a.im;
  }
}

// External wavefunctions, exported for the explicit-colour cross-check.
// kind 0: u, 1: v, 2: ubar (=u^dagger gamma^0), 3: vbar, 4: eps (incoming), 5: eps* (outgoing)
void or_wavefunction(int kind, const double* p, double m, int lam, double* out /* 8 */) {
  P4<double> P{p[0], p[1], p[2], p[3]};
  C4<double> w;
  switch (kind) {
    case 0: w = uspinor(P, m, lam); break;
    case 1: w = vspinor(P, m, lam); break;
    case 2: w = dbar(uspinor(P, m, lam)); break;
    case 3: w = dbar(vspinor(P, m, lam)); break;
    case 4: w = polvec(P, lam, false); break;
    default: w = polvec(P, lam, true); break;
  }
  for (int i = 0; i < 4; ++i) { out[2 * i] = w.c[i].re; out[2 * i + 1] = w.c[i].im; }
}

void or_gamma(double* re, double* im) {
  std::memcpy(re, GAM.re, sizeof(GAM.re));
  std::memcpy(im, GAM.im, sizeof(GAM.im));
}

double or_me_qqbar(const double* mom, double mt) {
  P4<double> p[4];
  for (int i = 0; i < 4; ++i) p[i] = P4<double>{mom[4 * i], mom[4 * i + 1], mom[4 * i + 2], mom[4 * i + 3]};
  return me_qqbar<double>(p[0], p[1], p[2], p[3], mt);
}

// w(x) for x [n][d]; pass flags optional.
void or_integrand(int h, int64_t n, const double* x, double* w, int* pass, int nthreads) {
  const State& S = *g_states[h];
  const int ng = S.cfg.n_g;
  const int d = 3 * (ng + 2) - 2;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t e = 0; e < n; ++e)
    w[e] = integrand_T<double>(S, x + (size_t)e * d, S.cfg.m_t, 0, nullptr, pass ? pass + e : nullptr);
}

// Integrand and its derivative in direction dir (1: m_t, 2..9: theta).
void or_integrand_grad(int h, int64_t n, const double* x, int dir, double* w, double* dw, int nthreads) {
  const State& S = *g_states[h];
  const int ng = S.cfg.n_g;
  const int d = 3 * (ng + 2) - 2;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t e = 0; e < n; ++e) {
    Dual mt(S.cfg.m_t, dir == 1 ? 1.0 : 0.0);
    Dual r = integrand_T<Dual>(S, x + (size_t)e * d, mt, dir, nullptr, nullptr);
    w[e] = r.v;
    dw[e] = r.d;
  }
}

// Integrand with momenta output: mom [n][n_ext][4] (p1,p2,t,tb,gluons).
void or_integrand_mom(int h, int64_t n, const double* x, double* w, double* mom) {
  const State& S = *g_states[h];
  const int ng = S.cfg.n_g;
  const int d = 3 * (ng + 2) - 2;
  const int next = ng + 4;
  for (int64_t e = 0; e < n; ++e) {
    std::fill(mom + (size_t)e * next * 4, mom + (size_t)(e + 1) * next * 4, 0.0);
    w[e] = integrand_T<double>(S, x + (size_t)e * d, S.cfg.m_t, 0, mom + (size_t)e * next * 4, nullptr);
  }
}

// One VEGAS iteration of n events drawn from Philox with counters
// (event, iter, call, 0) and key (seed, purpose), mapped through edges.
// out[0] = sum w, out[1] = sum w^2 (Kahan-compensated); hist[d][nb] += w^2;
// counts[0] = events with w != 0; counts[1] = non-finite weights (dropped).
void or_vegas_iteration(int h, const double* edges, int nb, uint64_t iter, int64_t ev0, int64_t n, uint64_t seed,
                        uint64_t purpose, double* out, double* hist, int64_t* counts, int nthreads) {
  const State& S = *g_states[h];
  const int ng = S.cfg.n_g;
  const int d = 3 * (ng + 2) - 2;
  int nt = 1;
#ifdef _OPENMP
  nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
  std::vector<double> s1(nt, 0.0), c1(nt, 0.0), s2(nt, 0.0), c2(nt, 0.0);
  std::vector<double> hh((size_t)nt * d * nb, 0.0);
  std::vector<int64_t> nz(nt, 0), bad(nt, 0);
#ifdef _OPENMP
#pragma omp parallel num_threads(nt)
#endif
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
    std::vector<double> y(d), x(d);
    std::vector<int> bins(d);
    for (int64_t e = lo; e < hi; ++e) {
      event_uniforms((uint64_t)(ev0 + e), iter, seed, purpose, d, y.data());
      double jac = vegas_map(edges, d, nb, y.data(), x.data(), bins.data());
      double f = integrand_T<double>(S, x.data(), S.cfg.m_t, 0, nullptr, nullptr);
      double w = f * jac;
      if (!std::isfinite(w)) { bad[t]++; continue; }
      if (w != 0.0) nz[t]++;
      // Kahan
      double yk = w - c1[t], tk = s1[t] + yk;
      c1[t] = (tk - s1[t]) - yk;
      s1[t] = tk;
      double w2 = w * w;
      yk = w2 - c2[t]; tk = s2[t] + yk;
      c2[t] = (tk - s2[t]) - yk;
      s2[t] = tk;
      for (int j = 0; j < d; ++j) hh[(size_t)t * d * nb + (size_t)j * nb + bins[j]] += w2;
    }
  }
  double S1 = 0, S2 = 0;
  for (int t = 0; t < nt; ++t) { S1 += s1[t]; S2 += s2[t]; }
  out[0] = S1;
  out[1] = S2;
  for (int t = 0; t < nt; ++t)
    for (size_t i = 0; i < (size_t)d * nb; ++i) hist[i] += hh[(size_t)t * d * nb + i];
  counts[0] = 0; counts[1] = 0;
  for (int t = 0; t < nt; ++t) { counts[0] += nz[t]; counts[1] += bad[t]; }
}

// VEGAS iteration on an analytic test integrand: a product over d dimensions
// of normalised Gaussians of width sig centred at 0.5 (integral over the unit
// cube = erf(0.5/(sig sqrt2))^d), or f = 1 when sig <= 0.
void or_vegas_iteration_gauss(int d, double sig, const double* edges, int nb, uint64_t iter, int64_t n,
                              uint64_t seed, uint64_t purpose, double* out, double* hist) {
  std::vector<double> y(d), x(d);
  std::vector<int> bins(d);
  double s1 = 0, c1 = 0, s2 = 0, c2 = 0;
  for (int64_t e = 0; e < n; ++e) {
    event_uniforms((uint64_t)e, iter, seed, purpose, d, y.data());
    double jac = vegas_map(edges, d, nb, y.data(), x.data(), bins.data());
    double f = 1.0;
    if (sig > 0)
      for (int j = 0; j < d; ++j) {
        double z = (x[j] - 0.5) / sig;
        f *= std::exp(-0.5 * z * z) / (sig * std::sqrt(2.0 * M_PI));
      }
    double w = f * jac;
    double yk = w - c1, tk = s1 + yk;
    c1 = (tk - s1) - yk; s1 = tk;
    yk = w * w - c2; tk = s2 + yk;
    c2 = (tk - s2) - yk; s2 = tk;
    for (int j = 0; j < d; ++j) hist[(size_t)j * nb + bins[j]] += w * w;
  }
  out[0] = s1;
  out[1] = s2;
}

}  // extern "C"
