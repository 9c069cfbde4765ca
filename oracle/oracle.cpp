// CPU oracle for leading-order |M|^2 — TEST INFRASTRUCTURE ONLY.
//
// Only tests, the smoke check and the benchmark's CPU-baseline leg load this
// library.  It shares nothing with the GPU path: spinors are built in the
// Dirac representation (the GPU path uses the chiral one), amplitudes come
// from a colour-ordered Berends-Giele recursion (the GPU path sums Feynman
// diagrams built from HELAS-style vertex calls), and the colour matrix comes
// from brute-force sums over explicit Gell-Mann matrices.
//
// Physics inputs (the paper is silent on all formulas; it only names the
// processes validated against MG5_aMC in its Summary section and the
// restriction to LO QED/QCD):
//   * Feynman rules (Peskin-Schroeder), all vertex momenta incoming:
//       f fbar photon : -i e Q gamma^mu
//       f fbar Z      : -i e gamma^mu (cL P_L + cR P_R),
//                       cL = (T3 - Q s_W^2)/(s_W c_W), cR = -Q s_W^2/(s_W c_W)
//       q qbar g      : +i g_s gamma^mu t^a
//       g g g         : g_s f^{abc} [g^{mu nu}(k-p)^rho + g^{nu rho}(p-q)^mu
//                                    + g^{rho mu}(q-k)^nu]
//       g g g g       : -i g_s^2 [f^{abe}f^{cde}(g^{mu rho}g^{nu sigma} - g^{mu sigma}g^{nu rho})
//                                + f^{ace}f^{bde}(g^{mu nu}g^{rho sigma} - g^{mu sigma}g^{nu rho})
//                                + f^{ade}f^{bce}(g^{mu nu}g^{rho sigma} - g^{mu rho}g^{nu sigma})]
//     propagators: fermion i(p/+m)/(p^2-m^2+i m Gamma); gluon/photon -i g/p^2;
//     Z -i(g - p p/M^2)/(p^2-M^2+i M Gamma).
//   * Fixed-width scheme; optional zero width for t-channel top propagators
//     (the "zero-width t-channel mode" of the paper's Sec. 3, Tables 1-2).  A
//     propagator is t-channel when the external legs on one side of it contain
//     exactly one of the two incoming legs.
//   * Average over initial helicities and colours, 1/n! for n identical
//     final-state gluons.
#include "oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

template <class T> using cx = std::complex<T>;

template <class T> struct V4 { cx<T> c[4]; };   // contravariant 4-vector (complex allowed)
template <class T> struct Sp { cx<T> c[4]; };   // Dirac spinor, column or barred row
template <class T> struct M4 { cx<T> m[4][4]; };

// ------------------------------------------------------------------ algebra
template <class T> cx<T> mdot(const V4<T>& a, const V4<T>& b) {
  return a.c[0] * b.c[0] - a.c[1] * b.c[1] - a.c[2] * b.c[2] - a.c[3] * b.c[3];
}
template <class T> V4<T> vadd(const V4<T>& a, const V4<T>& b) {
  V4<T> r; for (int i = 0; i < 4; ++i) r.c[i] = a.c[i] + b.c[i]; return r;
}
template <class T> V4<T> vscale(const V4<T>& a, cx<T> s) {
  V4<T> r; for (int i = 0; i < 4; ++i) r.c[i] = a.c[i] * s; return r;
}
template <class T> V4<T> vzero() { V4<T> r; for (int i = 0; i < 4; ++i) r.c[i] = 0; return r; }
template <class T> V4<T> vreal(const T* p) { V4<T> r; for (int i = 0; i < 4; ++i) r.c[i] = p[i]; return r; }

// Dirac representation: gamma^0 = diag(1,1,-1,-1), gamma^k = [[0,s_k],[-s_k,0]],
// gamma^5 = [[0,1],[1,0]].
template <class T> struct Dirac {
  M4<T> g[4];
  M4<T> g5;
  Dirac() {
    const cx<T> I(0, 1);
    cx<T> s[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
    for (int mu = 0; mu < 4; ++mu)
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) g[mu].m[i][j] = 0;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) g5.m[i][j] = 0;
    g[0].m[0][0] = g[0].m[1][1] = 1;
    g[0].m[2][2] = g[0].m[3][3] = -1;
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          g[k + 1].m[a][2 + b] = s[k][a][b];
          g[k + 1].m[2 + a][b] = -s[k][a][b];
        }
    g5.m[0][2] = g5.m[1][3] = g5.m[2][0] = g5.m[3][1] = 1;
  }
};
template <class T> const Dirac<T>& dirac() { static const Dirac<T> d; return d; }

// V-slash = gamma^mu V_mu = V^0 g^0 - V^k g^k.
template <class T> M4<T> slash(const V4<T>& v) {
  const Dirac<T>& d = dirac<T>();
  M4<T> r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      r.m[i][j] = v.c[0] * d.g[0].m[i][j] - v.c[1] * d.g[1].m[i][j] - v.c[2] * d.g[2].m[i][j] -
                  v.c[3] * d.g[3].m[i][j];
  return r;
}
template <class T> Sp<T> row_mat(const Sp<T>& r, const M4<T>& m) {
  Sp<T> o;
  for (int j = 0; j < 4; ++j) {
    cx<T> s = 0;
    for (int i = 0; i < 4; ++i) s += r.c[i] * m.m[i][j];
    o.c[j] = s;
  }
  return o;
}
template <class T> Sp<T> mat_col(const M4<T>& m, const Sp<T>& c) {
  Sp<T> o;
  for (int i = 0; i < 4; ++i) {
    cx<T> s = 0;
    for (int j = 0; j < 4; ++j) s += m.m[i][j] * c.c[j];
    o.c[i] = s;
  }
  return o;
}
template <class T> cx<T> row_col(const Sp<T>& r, const Sp<T>& c) {
  cx<T> s = 0;
  for (int i = 0; i < 4; ++i) s += r.c[i] * c.c[i];
  return s;
}
template <class T> Sp<T> sp_scale(const Sp<T>& a, cx<T> s) {
  Sp<T> r; for (int i = 0; i < 4; ++i) r.c[i] = a.c[i] * s; return r;
}
template <class T> Sp<T> sp_add(const Sp<T>& a, const Sp<T>& b) {
  Sp<T> r; for (int i = 0; i < 4; ++i) r.c[i] = a.c[i] + b.c[i]; return r;
}
template <class T> Sp<T> sp_zero() { Sp<T> r; for (int i = 0; i < 4; ++i) r.c[i] = 0; return r; }
// Current r gamma^mu c (upper index).
template <class T> V4<T> sandwich(const Sp<T>& r, const Sp<T>& c) {
  const Dirac<T>& d = dirac<T>();
  V4<T> j;
  for (int mu = 0; mu < 4; ++mu) j.c[mu] = row_col(r, mat_col(d.g[mu], c));
  return j;
}
template <class T> Sp<T> chiral_proj(const Sp<T>& c, int sign /* -1: P_L, +1: P_R */) {
  const Dirac<T>& d = dirac<T>();
  Sp<T> g5c = mat_col(d.g5, c);
  Sp<T> r;
  for (int i = 0; i < 4; ++i) r.c[i] = (c.c[i] + T(sign) * g5c.c[i]) * T(0.5);
  return r;
}

// ------------------------------------------------------------ external states
// Polar angles of the 3-momentum; phi = 0 on the z axis.
template <class T> void angles(const T* p, T& theta, T& phi) {
  T pt = std::sqrt(p[1] * p[1] + p[2] * p[2]);
  theta = std::atan2(pt, p[3]);
  phi = (pt > 0) ? std::atan2(p[2], p[1]) : T(0);
}
// Two-component helicity eigenstates of sigma.p_hat (eigenvalue lam).
template <class T> void chi(const T* p, int lam, cx<T>* x) {
  T th, ph;
  angles(p, th, ph);
  T c = std::cos(th / 2), s = std::sin(th / 2);
  cx<T> e(std::cos(ph), std::sin(ph));
  if (lam > 0) { x[0] = c; x[1] = e * s; }
  else { x[0] = -std::conj(e) * s; x[1] = c; }
}
template <class T> T pabs(const T* p) { return std::sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]); }
// Dirac-representation spinors: u = (sqrt(E+m) chi ; lam|p|/sqrt(E+m) chi),
// v = (-lam|p|/sqrt(E+m) chi_{-lam} ; sqrt(E+m) chi_{-lam}).
template <class T> Sp<T> spinor_u(const T* p, T m, int lam) {
  cx<T> x[2]; chi(p, lam, x);
  T a = std::sqrt(p[0] + m), b = T(lam) * pabs(p) / a;
  Sp<T> u; u.c[0] = a * x[0]; u.c[1] = a * x[1]; u.c[2] = b * x[0]; u.c[3] = b * x[1];
  return u;
}
template <class T> Sp<T> spinor_v(const T* p, T m, int lam) {
  cx<T> x[2]; chi(p, -lam, x);
  T a = std::sqrt(p[0] + m), b = -T(lam) * pabs(p) / a;
  Sp<T> v; v.c[0] = b * x[0]; v.c[1] = b * x[1]; v.c[2] = a * x[0]; v.c[3] = a * x[1];
  return v;
}
// Dirac adjoint psi^dagger gamma^0, stored as a row.
template <class T> Sp<T> bar(const Sp<T>& s) {
  Sp<T> r;
  r.c[0] = std::conj(s.c[0]); r.c[1] = std::conj(s.c[1]);
  r.c[2] = -std::conj(s.c[2]); r.c[3] = -std::conj(s.c[3]);
  return r;
}
// Massless vector polarisation eps(k, lam) = (-lam e1 - i e2)/sqrt2 with
// e1 = (0, cos th cos ph, cos th sin ph, -sin th), e2 = (0, -sin ph, cos ph, 0).
template <class T> V4<T> polvec(const T* k, int lam) {
  T th, ph;
  angles(k, th, ph);
  T e1[4] = {0, std::cos(th) * std::cos(ph), std::cos(th) * std::sin(ph), -std::sin(th)};
  T e2[4] = {0, -std::sin(ph), std::cos(ph), 0};
  const T r2 = std::sqrt(T(2));
  V4<T> e;
  for (int i = 0; i < 4; ++i) e.c[i] = cx<T>(-T(lam) * e1[i], -e2[i]) / r2;
  return e;
}
template <class T> V4<T> vconj(const V4<T>& a) {
  V4<T> r; for (int i = 0; i < 4; ++i) r.c[i] = std::conj(a.c[i]); return r;
}

// --------------------------------------------------------------- parameters
template <class T> struct Couplings {
  T e, gs, cl, cr, mz, wz, mt, wt;
  bool tzero;
  explicit Couplings(const oracle_params& p) {
    const T pi = std::acos(T(-1));
    e = std::sqrt(4 * pi * T(p.alpha_em));
    gs = std::sqrt(4 * pi * T(p.alpha_s));
    T s2 = T(p.sin2w), sw = std::sqrt(s2), cw = std::sqrt(1 - s2);
    const T Q = -1, T3 = T(-0.5);
    cl = (T3 - Q * s2) / (sw * cw);
    cr = (-Q * s2) / (sw * cw);
    mz = T(p.mz); wz = T(p.wz); mt = T(p.mt); wt = T(p.wt);
    tzero = p.tchan_zero_width != 0;
  }
};

// light quark-antiquark annihilation into t tbar (processes 5 and 6)
bool is_qq(int proc) { return proc == 5 || proc == 6; }
// one light-quark line, t tbar and one gluon (processes 7..12)
bool is_qqg(int proc) { return proc >= 7 && proc <= 12; }
int npar_of(int proc) {
  if (proc == 0 || is_qq(proc)) return 4;
  if (is_qqg(proc)) return 5;
  return proc >= 1 && proc <= 4 ? 3 + proc : -1;
}
int ngluon_of(int proc) { return proc >= 1 && proc <= 4 ? proc + 1 : 0; }
long factorial(int n) { long f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }
double iden_of(int proc) {
  if (proc == 0) return 4.0;
  if (is_qq(proc)) return 36.0;   // 2 x 2 spins, 3 x 3 colours
  if (proc == 7 || proc == 8) return 36.0;
  if (is_qqg(proc)) return 96.0;  // quark (or antiquark) and gluon in: 2 x 2 spins, 3 x 8 colours
  int nfinal_g = ngluon_of(proc) - 2;
  return 256.0 * double(factorial(nfinal_g));
}

// ------------------------------------------------------------- ee -> mumu
// Legs: 0 e+ (incoming antifermion, vbar), 1 e- (incoming fermion, u),
//       2 mu+ (outgoing antifermion, v), 3 mu- (outgoing fermion, ubar).
template <class T> cx<T> amp_eemumu(const Couplings<T>& c, const T (*p)[4], int hel) {
  int lam[4];
  for (int i = 0; i < 4; ++i) lam[i] = ((hel >> i) & 1) ? 1 : -1;
  Sp<T> vb0 = bar(spinor_v(p[0], T(0), lam[0]));
  Sp<T> u1 = spinor_u(p[1], T(0), lam[1]);
  Sp<T> v2 = spinor_v(p[2], T(0), lam[2]);
  Sp<T> ub3 = bar(spinor_u(p[3], T(0), lam[3]));
  const cx<T> I(0, 1);
  const T Q = -1;
  T q[4];
  for (int i = 0; i < 4; ++i) q[i] = p[0][i] + p[1][i];
  V4<T> qv = vreal<T>(q);
  T s = q[0] * q[0] - q[1] * q[1] - q[2] * q[2] - q[3] * q[3];
  // photon: vertex -ieQ gamma^mu twice, propagator -i g_{mu nu}/s
  V4<T> j1 = sandwich(vb0, u1), j2 = sandwich(ub3, v2);
  cx<T> m_gam = (-I * c.e * Q) * (-I * c.e * Q) * (-I / s) * mdot(j1, j2);
  // Z: vertex -ie gamma^mu (cL P_L + cR P_R), unitary-gauge propagator
  V4<T> z1 = vadd(vscale(sandwich(vb0, chiral_proj(u1, -1)), cx<T>(c.cl)),
                  vscale(sandwich(vb0, chiral_proj(u1, +1)), cx<T>(c.cr)));
  V4<T> z2 = vadd(vscale(sandwich(ub3, chiral_proj(v2, -1)), cx<T>(c.cl)),
                  vscale(sandwich(ub3, chiral_proj(v2, +1)), cx<T>(c.cr)));
  cx<T> den = T(1) / cx<T>(s - c.mz * c.mz, c.mz * c.wz);
  cx<T> contr = mdot(z1, z2) - mdot(z1, qv) * mdot(z2, qv) / (c.mz * c.mz);
  cx<T> m_z = (-I * c.e) * (-I * c.e) * (-I) * den * contr;
  return m_gam + m_z;
}

// ------------------------------------------------------- q qbar -> t tbar
// Process 5 "u u~ > t t~": legs 0 q (incoming, u), 1 qbar (incoming, vbar),
// 2 t (outgoing, ubar), 3 tbar (outgoing, v); process 6 "u~ u > t t~" has
// the incoming legs in the other order.  One diagram, the s-channel gluon:
//   M = A * sum_a (t^a)_{c_qbar c_q} (t^a)_{c_t c_tbar},
//   A = [vbar gamma^mu u] (-i g)^2 (-i g_{mu nu} / s) [ubar gamma^nu v].
template <class T> cx<T> amp_qqtt(const Couplings<T>& c, const T (*p)[4], int hel, int iq, int iqb) {
  int lam[4];
  for (int i = 0; i < 4; ++i) lam[i] = ((hel >> i) & 1) ? 1 : -1;
  Sp<T> u = spinor_u(p[iq], T(0), lam[iq]);
  Sp<T> vb = bar(spinor_v(p[iqb], T(0), lam[iqb]));
  Sp<T> ub = bar(spinor_u(p[2], c.mt, lam[2]));
  Sp<T> v = spinor_v(p[3], c.mt, lam[3]);
  T q[4];
  for (int i = 0; i < 4; ++i) q[i] = p[0][i] + p[1][i];
  const T s = q[0] * q[0] - q[1] * q[1] - q[2] * q[2] - q[3] * q[3];
  const cx<T> I(0, 1);
  return (-I * c.gs) * (-I * c.gs) * (-I / s) * mdot(sandwich(vb, u), sandwich(ub, v));
}

// ------------------------------------- light-quark line + t tbar + one gluon
// Processes 7 "u u~ > t t~ g", 8 "u~ u > t t~ g", 9 "u g > t t~ u",
// 10 "g u > t t~ u", 11 "u~ g > t t~ u~", 12 "g u~ > t t~ u~" (massless u).
// The light line runs along the fermion arrow from its column end (u(p) of
// an incoming quark or v(p) of an outgoing antiquark) to its row end (ubar(p)
// of an outgoing quark or vbar(p) of an incoming antiquark); the top line
// from v(p3) to ubar(p2).  Literal Feynman rules: quark-gluon vertex
// -i g gamma^mu t^a, fermion propagator i(P/ + m)/(P^2 - m^2 + i m Gamma),
// gluon propagator -i g_{mu nu}/Q^2, three-gluon vertex
// -g f^{abc} [g^{mu nu}(k1-k2)^rho + g^{nu rho}(k2-k3)^mu + g^{rho mu}(k3-k1)^nu]
// (all momenta incoming).  Five diagrams: the gluon on the light line at its
// column or row end, on the top line at the t or tbar end, or on the gluon
// exchanged between the lines.
struct QqgLegs { int col, row, glu; bool col_in, row_in, glu_in; };
QqgLegs qqg_legs(int proc) {
  switch (proc) {
    case 7: return {0, 1, 4, true, true, false};
    case 8: return {1, 0, 4, true, true, false};
    case 9: return {0, 4, 1, true, false, true};
    case 10: return {1, 4, 0, true, false, true};
    case 11: return {4, 0, 1, false, true, true};
    default: return {4, 1, 0, false, true, true};
  }
}

// Diagram-basis colour factors for explicit colours (r, c of the light line's
// row and column ends, t, tb of the top line's, b of the gluon) and the 5x5
// matrix sum_colours conj(c_D) c_D', by brute force.
const std::vector<std::complex<long double>>& qqg_colour_matrix();

template <class T> M4<T> m4_scale(const M4<T>& a, cx<T> s) {
  M4<T> r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) r.m[i][j] = a.m[i][j] * s;
  return r;
}
template <class T> M4<T> m4_add_diag(const M4<T>& a, cx<T> s) {
  M4<T> r = a;
  for (int i = 0; i < 4; ++i) r.m[i][i] += s;
  return r;
}
template <class T> T msq4(const T* k) { return k[0] * k[0] - k[1] * k[1] - k[2] * k[2] - k[3] * k[3]; }

// Lorentz parts A_D of the five diagrams for helicity hel; gauge: replace the
// gluon polarisation by k/k^0.
template <class T>
void qqg_diagrams(const Couplings<T>& c, const T (*p)[4], int proc, int hel, bool gauge, cx<T>* A) {
  const QqgLegs L = qqg_legs(proc);
  int lam[5];
  for (int i = 0; i < 5; ++i) lam[i] = ((hel >> i) & 1) ? 1 : -1;
  const cx<T> I(0, 1);
  const T g = c.gs;
  // external states
  const Sp<T> colL = L.col_in ? spinor_u(p[L.col], T(0), lam[L.col]) : spinor_v(p[L.col], T(0), lam[L.col]);
  const Sp<T> rowL = L.row_in ? bar(spinor_v(p[L.row], T(0), lam[L.row])) : bar(spinor_u(p[L.row], T(0), lam[L.row]));
  const Sp<T> rowT = bar(spinor_u(p[2], c.mt, lam[2]));
  const Sp<T> colT = spinor_v(p[3], c.mt, lam[3]);
  V4<T> eps;
  if (gauge) {
    for (int m = 0; m < 4; ++m) eps.c[m] = p[L.glu][m] / p[L.glu][0];
  } else {
    eps = polvec(p[L.glu], lam[L.glu]);
    if (!L.glu_in) eps = vconj(eps);
  }
  // momenta flowing into the diagram
  T qc[4], qr[4], kg[4], qt[4], qtb[4];
  for (int m = 0; m < 4; ++m) {
    qc[m] = L.col_in ? p[L.col][m] : -p[L.col][m];
    qr[m] = L.row_in ? p[L.row][m] : -p[L.row][m];
    kg[m] = L.glu_in ? p[L.glu][m] : -p[L.glu][m];
    qt[m] = -p[2][m];
    qtb[m] = -p[3][m];
  }
  auto vtx = [&](const V4<T>& v) { return m4_scale(slash(v), -I * g); };          // -i g V/
  auto fprop = [&](const T* P, T m, T w) {                                         // i(P/ + m)/(P^2 - m^2 + i m w)
    const cx<T> den = cx<T>(msq4(P) - m * m, m * w);
    return m4_scale(m4_add_diag(slash(vreal<T>(P)), cx<T>(m)), I / den);
  };
  auto gprop = [&](const T* Q) { return -I / msq4(Q); };
  // t-channel top propagator: the legs on one side hold exactly one incoming leg
  const T wtop = (c.tzero && L.glu_in) ? T(0) : c.wt;
  // currents
  const V4<T> JT = vscale(sandwich(rowT, colT), -I * g);
  const V4<T> JL = vscale(sandwich(rowL, colL), -I * g);
  T Q0[4], P1[4], P2[4], PT3[4], PT4[4], QT[4];
  for (int m = 0; m < 4; ++m) {
    Q0[m] = qc[m] + qr[m];            // gluon from the light line (no extra gluon on it)
    P1[m] = qc[m] + kg[m];            // D1: along the arrow after absorbing the gluon at the column end
    P2[m] = -qr[m] - kg[m];           // D2: along the arrow before the gluon at the row end
    PT3[m] = -qt[m] - kg[m];          // D3: top line, gluon at the t end
    PT4[m] = qtb[m] + kg[m];          // D4: top line, gluon at the tbar end
    QT[m] = qt[m] + qtb[m];           // gluon into the top line's vertex from the top side
  }
  T Q1[4];
  for (int m = 0; m < 4; ++m) Q1[m] = qc[m] + qr[m] + kg[m];
  // D1, D2: gluon on the light line; exchanged gluon carries Q1
  {
    const Sp<T> s1 = mat_col(fprop(P1, T(0), T(0)), mat_col(vtx(eps), colL));
    const V4<T> J1 = vscale(sandwich(rowL, s1), -I * g);
    A[0] = mdot(J1, JT) * gprop(Q1);
    const Sp<T> r2 = row_mat(row_mat(rowL, vtx(eps)), fprop(P2, T(0), T(0)));
    const V4<T> J2 = vscale(sandwich(r2, colL), -I * g);
    A[1] = mdot(J2, JT) * gprop(Q1);
  }
  // D3, D4: gluon on the top line; exchanged gluon carries Q0
  {
    const Sp<T> r3 = row_mat(row_mat(rowT, vtx(eps)), fprop(PT3, c.mt, wtop));
    const V4<T> J3 = vscale(sandwich(r3, colT), -I * g);
    A[2] = mdot(JL, J3) * gprop(Q0);
    const Sp<T> s4 = mat_col(fprop(PT4, c.mt, wtop), mat_col(vtx(eps), colT));
    const V4<T> J4 = vscale(sandwich(rowT, s4), -I * g);
    A[3] = mdot(JL, J4) * gprop(Q0);
  }
  // D5: three-gluon vertex (a = light-line gluon with Q0, b = external gluon
  // with kg, c = top-line gluon with QT; all into the vertex)
  {
    const V4<T> JLp = vscale(JL, gprop(Q0)), JTp = vscale(JT, gprop(QT));
    V4<T> d12, d23, d31;
    for (int m = 0; m < 4; ++m) {
      d12.c[m] = Q0[m] - kg[m];
      d23.c[m] = kg[m] - QT[m];
      d31.c[m] = QT[m] - Q0[m];
    }
    A[4] = -g * (mdot(JLp, eps) * mdot(d12, JTp) + mdot(eps, JTp) * mdot(d23, JLp) + mdot(JTp, JLp) * mdot(d31, eps));
  }
}

template <class T> T qqg_me_hel(const Couplings<T>& c, const T (*p)[4], int proc, int hel, bool gauge) {
  cx<T> A[5];
  qqg_diagrams(c, p, proc, hel, gauge, A);
  const auto& C = qqg_colour_matrix();
  T sum = 0;
  for (int d = 0; d < 5; ++d)
    for (int e = 0; e < 5; ++e) {
      const std::complex<long double> cde = C[size_t(d) * 5 + e];
      sum += (std::conj(A[d]) * cx<T>(T(cde.real()), T(cde.imag())) * A[e]).real();
    }
  return sum;
}

// ------------------------------------------------------------------- QCD
// Legs: 0,1 incoming gluons; 2 t (outgoing, ubar); 3 tbar (outgoing, v);
// 4.. outgoing gluons.  Gluon g (0-based) sits on leg gl(g).
inline int gluon_leg(int g) { return g < 2 ? g : g + 2; }

template <class T> struct QcdEvent {
  int ng;
  T k[5][4];        // momentum flowing INTO the diagram along each gluon
  V4<T> eps[5];     // eps for incoming, eps* for outgoing gluons
  Sp<T> ubar_t, v_tb;
  T pt[4];          // outgoing top momentum
};

template <class T>
QcdEvent<T> qcd_setup(const Couplings<T>& c, const T (*p)[4], int ng, int hel, int gauge_leg) {
  QcdEvent<T> ev;
  ev.ng = ng;
  for (int g = 0; g < ng; ++g) {
    int leg = gluon_leg(g);
    int lam = ((hel >> leg) & 1) ? 1 : -1;
    T sgn = leg < 2 ? T(1) : T(-1);
    for (int i = 0; i < 4; ++i) ev.k[g][i] = sgn * p[leg][i];
    if (leg == gauge_leg) {
      V4<T> kv = vreal<T>(p[leg]);
      ev.eps[g] = vscale(kv, cx<T>(T(1) / p[leg][0]));
    } else {
      V4<T> e = polvec(p[leg], lam);
      ev.eps[g] = leg < 2 ? e : vconj(e);
    }
  }
  int lt = ((hel >> 2) & 1) ? 1 : -1, ltb = ((hel >> 3) & 1) ? 1 : -1;
  ev.ubar_t = bar(spinor_u(p[2], c.mt, lt));
  ev.v_tb = spinor_v(p[3], c.mt, ltb);
  for (int i = 0; i < 4; ++i) ev.pt[i] = p[2][i];
  return ev;
}

// Lorentz part of the three-gluon vertex contracted with currents a and b
// that carry momenta ka and kb into the vertex; the free index belongs to the
// third leg, whose incoming momentum is -(ka+kb).  Colour f^{x a b}.
template <class T> V4<T> vvv(const V4<T>& ja, const T* ka, const V4<T>& jb, const T* kb) {
  T kx[4], kxa[4], pab[4], qbx[4];
  for (int i = 0; i < 4; ++i) {
    kx[i] = -(ka[i] + kb[i]);
    kxa[i] = kx[i] - ka[i];   // (k - p)
    pab[i] = ka[i] - kb[i];   // (p - q)
    qbx[i] = kb[i] - kx[i];   // (q - k)
  }
  cx<T> t1 = mdot(vreal<T>(kxa), jb), t2 = mdot(ja, jb), t3 = mdot(vreal<T>(qbx), ja);
  V4<T> r;
  for (int mu = 0; mu < 4; ++mu) r.c[mu] = ja.c[mu] * t1 + t2 * pab[mu] + jb.c[mu] * t3;
  return r;
}

template <class T> cx<T> msq(const T* k) {
  return cx<T>(k[0] * k[0] - k[1] * k[1] - k[2] * k[2] - k[3] * k[3], 0);
}

// Top propagator i(P/+m)/(P^2 - m^2 + i m Gamma) applied from the right to a
// row spinor; P is the momentum along the fermion-number arrow.
template <class T>
Sp<T> prop_row(const Sp<T>& r, const T* P, const Couplings<T>& c, bool tchan) {
  const cx<T> I(0, 1);
  T w = (tchan && c.tzero) ? T(0) : c.wt;
  cx<T> den = cx<T>(P[0] * P[0] - P[1] * P[1] - P[2] * P[2] - P[3] * P[3] - c.mt * c.mt, c.mt * w);
  M4<T> num = slash(vreal<T>(P));
  for (int i = 0; i < 4; ++i) num.m[i][i] += c.mt;
  return sp_scale(row_mat(r, num), I / den);
}

// Colour-ordered partial amplitudes A(sigma) for every ordering sigma of the
// gluons along the top line, c_sigma = (t^{a_s1}...t^{a_sn})_{i_t j_tbar}.
// Derived from the literal rules with f^{xbc} t^x = -i[t^b, t^c]:
//   ordered 3-gluon vertex  : -i g V(J_A, J_B)
//   ordered 4-gluon vertex  : -i g^2 [J_A (J_B.J_C) + J_C (J_A.J_B) - 2 J_B (J_A.J_C)]
//   gluon propagator        : -i / K^2
//   quark-gluon vertex      : +i g gamma^mu (colour coefficient 1)
template <class T>
void partial_amps(const Couplings<T>& c, const QcdEvent<T>& ev, cx<T>* A) {
  const int n = ev.ng;
  const cx<T> I(0, 1);
  const T g = c.gs;
  int perm[5];
  for (int i = 0; i < n; ++i) perm[i] = i;
  long idx = 0;
  do {
    V4<T> J[5][5];
    T K[5][5][4];
    for (int i = 0; i < n; ++i) {
      J[i][i] = ev.eps[perm[i]];
      for (int m = 0; m < 4; ++m) K[i][i][m] = ev.k[perm[i]][m];
    }
    for (int len = 2; len <= n; ++len) {
      for (int i = 0; i + len - 1 < n; ++i) {
        int j = i + len - 1;
        for (int m = 0; m < 4; ++m) K[i][j][m] = K[i][j - 1][m] + K[j][j][m];
        V4<T> acc = vzero<T>();
        for (int m = i; m < j; ++m)
          acc = vadd(acc, vscale(vvv(J[i][m], K[i][m], J[m + 1][j], K[m + 1][j]), -I * g));
        for (int m = i; m < j; ++m)
          for (int l = m + 1; l < j; ++l) {
            const V4<T>& a = J[i][m];
            const V4<T>& b = J[m + 1][l];
            const V4<T>& cc = J[l + 1][j];
            cx<T> bc = mdot(b, cc), ab = mdot(a, b), ac = mdot(a, cc);
            V4<T> x;
            for (int mu = 0; mu < 4; ++mu)
              x.c[mu] = a.c[mu] * bc + cc.c[mu] * ab - T(2) * b.c[mu] * ac;
            acc = vadd(acc, vscale(x, -I * g * g));
          }
        J[i][j] = vscale(acc, -I / msq(K[i][j]));
      }
    }
    // Row currents along the top line: U[j] has absorbed gluons perm[0..j-1].
    Sp<T> U[5];
    U[0] = ev.ubar_t;
    for (int j = 1; j < n; ++j) {
      T P[4];
      int nin = 0;  // incoming legs on the top side of this propagator
      for (int m = 0; m < 4; ++m) P[m] = ev.pt[m];
      for (int l = 0; l < j; ++l) {
        for (int m = 0; m < 4; ++m) P[m] -= ev.k[perm[l]][m];
        if (gluon_leg(perm[l]) < 2) ++nin;
      }
      Sp<T> s = sp_zero<T>();
      for (int i = 0; i < j; ++i)
        s = sp_add(s, row_mat(U[i], slash(vscale(J[i][j - 1], I * g))));
      U[j] = prop_row(s, P, c, nin == 1);
    }
    cx<T> a = 0;
    for (int i = 0; i < n; ++i) a += row_col(row_mat(U[i], slash(vscale(J[i][n - 1], I * g))), ev.v_tb);
    A[idx++] = a;
  } while (std::next_permutation(perm, perm + n));
}

// --------------------------------------------------------------- SU(3)
// R is the real type of the entries: double for the colour-dressed pins,
// long double for the colour matrices, whose rounding would otherwise bound
// the long-double evaluation's accuracy on events where the colour sum
// cancels strongly.
template <class R> struct SU3T {
  std::complex<R> t[8][3][3];
  R f[8][8][8];
  SU3T() {
    typedef std::complex<R> C;
    const C I(0, 1);
    for (int a = 0; a < 8; ++a)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[a][i][j] = 0;
    t[0][0][1] = t[0][1][0] = 1;
    t[1][0][1] = -I; t[1][1][0] = I;
    t[2][0][0] = 1; t[2][1][1] = -1;
    t[3][0][2] = t[3][2][0] = 1;
    t[4][0][2] = -I; t[4][2][0] = I;
    t[5][1][2] = t[5][2][1] = 1;
    t[6][1][2] = -I; t[6][2][1] = I;
    const R r3 = R(1) / std::sqrt(R(3));
    t[7][0][0] = r3; t[7][1][1] = r3; t[7][2][2] = -2 * r3;
    for (int a = 0; a < 8; ++a)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[a][i][j] *= R(0.5);
    // f^{abc} = -2 i Tr(t^a [t^b, t^c])
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b)
        for (int c = 0; c < 8; ++c) {
          C tr = 0;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              for (int k = 0; k < 3; ++k)
                tr += t[a][i][j] * (t[b][j][k] * t[c][k][i] - t[c][j][k] * t[b][k][i]);
          R v = (R(-2) * I * tr).real();
          f[a][b][c] = std::fabs(v) < R(1e-14) ? R(0) : v;
        }
  }
};
using SU3 = SU3T<double>;
const SU3& su3() { static const SU3 s; return s; }
const SU3T<long double>& su3l() { static const SU3T<long double> s; return s; }

// c_sigma for explicit colours.
void colour_basis_values(int n, const int* col, std::complex<double>* out) {
  const SU3& s = su3();
  int perm[5];
  for (int i = 0; i < n; ++i) perm[i] = i;
  int it = col[n], jt = col[n + 1];
  long idx = 0;
  do {
    std::complex<double> row[3] = {0, 0, 0};
    row[it] = 1;
    for (int l = 0; l < n; ++l) {
      std::complex<double> nr[3] = {0, 0, 0};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) nr[j] += row[i] * s.t[col[perm[l]]][i][j];
      for (int j = 0; j < 3; ++j) row[j] = nr[j];
    }
    out[idx++] = row[jt];
  } while (std::next_permutation(perm, perm + n));
}

// C[sigma][tau] = sum_{a_1..a_n} Tr(P_sigma^dagger P_tau), P = t^{a_s1}...t^{a_sn}.
std::vector<long double> colour_matrix_brute(int n) {
  const SU3T<long double>& s = su3l();
  const int nf = int(factorial(n));
  long nassign = 1;
  for (int i = 0; i < n; ++i) nassign *= 8;
  std::vector<std::vector<int>> perms;
  {
    std::vector<int> p(n);
    for (int i = 0; i < n; ++i) p[i] = i;
    do perms.push_back(p); while (std::next_permutation(p.begin(), p.end()));
  }
  std::vector<std::complex<long double>> C(size_t(nf) * nf, 0.0);
  std::mutex mtx;
#pragma omp parallel
  {
    std::vector<std::complex<long double>> Cl(size_t(nf) * nf, 0.0);
    std::vector<std::complex<long double>> P(size_t(nf) * 9);
#pragma omp for schedule(dynamic)
    for (long as = 0; as < nassign; ++as) {
      int a[5];
      long r = as;
      for (int i = 0; i < n; ++i) { a[i] = int(r % 8); r /= 8; }
      for (int si = 0; si < nf; ++si) {
        std::complex<long double> M[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int l = 0; l < n; ++l) {
          std::complex<long double> N[3][3];
          const auto& tm = s.t[a[perms[si][l]]];
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
              N[i][j] = M[i][0] * tm[0][j] + M[i][1] * tm[1][j] + M[i][2] * tm[2][j];
          std::memcpy(M, N, sizeof(M));
        }
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) P[size_t(si) * 9 + i * 3 + j] = M[i][j];
      }
      for (int si = 0; si < nf; ++si)
        for (int ti = 0; ti < nf; ++ti) {
          std::complex<long double> acc = 0;
          for (int q = 0; q < 9; ++q) acc += std::conj(P[size_t(si) * 9 + q]) * P[size_t(ti) * 9 + q];
          Cl[size_t(si) * nf + ti] += acc;
        }
    }
    std::lock_guard<std::mutex> lk(mtx);
    for (size_t q = 0; q < C.size(); ++q) C[q] += Cl[q];
  }
  std::vector<long double> out(C.size());
  for (size_t q = 0; q < C.size(); ++q) out[q] = C[q].real();
  return out;
}

// sum over all colours of |sum_a (t^a)_{j i} (t^a)_{k l}|^2 (the colour
// factor of q qbar -> t tbar), by brute force
long double qq_colour_factor() {
  static const long double v = [] {
    const SU3T<long double>& s = su3l();
    long double acc = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) {
            std::complex<long double> x = 0;
            for (int a = 0; a < 8; ++a) x += s.t[a][j][i] * s.t[a][k][l];
            acc += std::norm(x);
          }
    return acc;
  }();
  return v;
}

// Colour factors of the five light-line + gluon diagrams for explicit
// colours, c_D = (t^a t^b)_{rc}(t^a)_{t tb}, (t^b t^a)_{rc}(t^a)_{t tb},
// (t^a)_{rc}(t^b t^a)_{t tb}, (t^a)_{rc}(t^a t^b)_{t tb}, f^{abc'}(t^a)_{rc}(t^c')_{t tb}
// (summed over a, c'), and M_{DE} = sum over r, c, t, tb, b of conj(c_D) c_E.
const std::vector<std::complex<long double>>& qqg_colour_matrix() {
  static const std::vector<std::complex<long double>> M = [] {
    const SU3T<long double>& s = su3l();
    std::vector<std::complex<long double>> m(25, 0.0L);
    auto prod = [&](int a, int b, int i, int j) {
      std::complex<long double> x = 0;
      for (int k = 0; k < 3; ++k) x += s.t[a][i][k] * s.t[b][k][j];
      return x;
    };
    for (int r = 0; r < 3; ++r)
      for (int cl = 0; cl < 3; ++cl)
        for (int t = 0; t < 3; ++t)
          for (int tb = 0; tb < 3; ++tb)
            for (int b = 0; b < 8; ++b) {
              std::complex<long double> f[5] = {0, 0, 0, 0, 0};
              for (int a = 0; a < 8; ++a) {
                f[0] += prod(a, b, r, cl) * s.t[a][t][tb];
                f[1] += prod(b, a, r, cl) * s.t[a][t][tb];
                f[2] += s.t[a][r][cl] * prod(b, a, t, tb);
                f[3] += s.t[a][r][cl] * prod(a, b, t, tb);
                for (int c2 = 0; c2 < 8; ++c2) f[4] += s.f[a][b][c2] * s.t[a][r][cl] * s.t[c2][t][tb];
              }
              for (int d = 0; d < 5; ++d)
                for (int e = 0; e < 5; ++e) m[size_t(d) * 5 + e] += std::conj(f[d]) * f[e];
            }
    return m;
  }();
  return M;
}

const std::vector<long double>& colour_matrix_cached(int n) {
  static std::mutex mtx;
  static std::vector<long double> cache[6];
  std::lock_guard<std::mutex> lk(mtx);
  if (cache[n].empty()) cache[n] = colour_matrix_brute(n);
  return cache[n];
}

// Colour-dressed amplitude: literal rules with explicit colour indices, the
// sum over all tree diagrams organised as a recursion over gluon subsets.
template <class T>
cx<T> dressed_amp(const Couplings<T>& c, const QcdEvent<T>& ev, const int* col) {
  const SU3& s = su3();
  const int n = ev.ng;
  const int full = (1 << n) - 1;
  const cx<T> I(0, 1);
  const T g = c.gs;
  std::vector<V4<T>> JD(size_t(full + 1) * 8);
  std::vector<std::array<T, 4>> K(full + 1);
  for (int S = 1; S <= full; ++S) {
    for (int m = 0; m < 4; ++m) {
      T acc = 0;
      for (int q = 0; q < n; ++q)
        if (S >> q & 1) acc += ev.k[q][m];
      K[S][m] = acc;
    }
  }
  auto J = [&](int S, int a) -> V4<T>& { return JD[size_t(S) * 8 + a]; };
  for (int S = 1; S <= full; ++S) {
    int pc = __builtin_popcount(S);
    if (pc == 1) {
      int q = __builtin_ctz(S);
      for (int a = 0; a < 8; ++a) J(S, a) = (a == col[q]) ? ev.eps[q] : vzero<T>();
      continue;
    }
    V4<T> acc[8];
    for (int a = 0; a < 8; ++a) acc[a] = vzero<T>();
    int low = S & (-S);
    // unordered binary splits {A, B}, A holds the lowest gluon
    for (int A = (S - 1) & S; A > 0; A = (A - 1) & S) {
      if (!(A & low)) continue;
      int B = S ^ A;
      for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
          for (int x = 0; x < 8; ++x) {
            double fv = s.f[x][a][b];
            if (fv == 0) continue;
            acc[x] = vadd(acc[x], vscale(vvv(J(A, a), K[A].data(), J(B, b), K[B].data()), cx<T>(g * T(fv))));
          }
        }
    }
    // unordered ternary splits {A, B, C}
    for (int A = (S - 1) & S; A > 0; A = (A - 1) & S) {
      if (!(A & low)) continue;
      int R = S ^ A;
      int lowR = R & (-R);
      for (int B = (R - 1) & R; B > 0; B = (B - 1) & R) {
        if (!(B & lowR)) continue;
        int Cs = R ^ B;
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b)
            for (int d = 0; d < 8; ++d) {
              const V4<T>& ja = J(A, a);
              const V4<T>& jb = J(B, b);
              const V4<T>& jc = J(Cs, d);
              cx<T> bc = mdot(jb, jc), ab = mdot(ja, jb), ac = mdot(ja, jc);
              for (int x = 0; x < 8; ++x) {
                double c1 = 0, c2 = 0, c3 = 0;
                for (int e = 0; e < 8; ++e) {
                  c1 += s.f[x][a][e] * s.f[b][d][e];
                  c2 += s.f[x][b][e] * s.f[a][d][e];
                  c3 += s.f[x][d][e] * s.f[a][b][e];
                }
                if (c1 == 0 && c2 == 0 && c3 == 0) continue;
                V4<T> v;
                for (int mu = 0; mu < 4; ++mu)
                  v.c[mu] = T(c1) * (jb.c[mu] * ac - jc.c[mu] * ab) +
                            T(c2) * (ja.c[mu] * bc - jc.c[mu] * ab) +
                            T(c3) * (ja.c[mu] * bc - jb.c[mu] * ac);
                acc[x] = vadd(acc[x], vscale(v, -I * g * g));
              }
            }
      }
    }
    for (int a = 0; a < 8; ++a) J(S, a) = vscale(acc[a], -I / msq(K[S].data()));
  }
  // top line: UD[S][i], S = gluons absorbed on the top side, open colour i
  std::vector<Sp<T>> UD(size_t(full + 1) * 3);
  auto U = [&](int S, int i) -> Sp<T>& { return UD[size_t(S) * 3 + i]; };
  for (int i = 0; i < 3; ++i) U(0, i) = (i == col[n]) ? ev.ubar_t : sp_zero<T>();
  auto attach = [&](int Sprev, int G, int j) {
    // sum_{i,x} U[Sprev][i] t^x_{ij} (i g J[G][x]/)
    Sp<T> r = sp_zero<T>();
    for (int x = 0; x < 8; ++x) {
      M4<T> sl = slash(vscale(J(G, x), I * g));
      for (int i = 0; i < 3; ++i) {
        std::complex<double> tc = s.t[x][i][j];
        if (tc == 0.0) continue;
        r = sp_add(r, sp_scale(row_mat(U(Sprev, i), sl), cx<T>(T(tc.real()), T(tc.imag()))));
      }
    }
    return r;
  };
  for (int S = 1; S < full; ++S) {
    T P[4];
    int nin = 0;
    for (int m = 0; m < 4; ++m) P[m] = ev.pt[m] - K[S][m];
    for (int q = 0; q < n; ++q)
      if ((S >> q & 1) && gluon_leg(q) < 2) ++nin;
    for (int j = 0; j < 3; ++j) {
      Sp<T> acc = sp_zero<T>();
      for (int G = S; G > 0; G = (G - 1) & S) acc = sp_add(acc, attach(S ^ G, G, j));
      U(S, j) = prop_row(acc, P, c, nin == 1);
    }
  }
  cx<T> m = 0;
  int jt = col[n + 1];
  for (int G = full; G > 0; G = (G - 1) & full) m += row_col(attach(full ^ G, G, jt), ev.v_tb);
  return m;
}

// Mass of leg i: the top quark and antiquark are legs 2 and 3 of every
// process but e+ e- -> mu+ mu-; every other external particle is massless.
double leg_mass(int proc, int i, double mt) { return proc != 0 && (i == 2 || i == 3) ? mt : 0.0; }

// External momenta on the mass shell.  |M|^2 is defined for on-shell
// momenta, and a double-precision input can only be on shell to rounding: its
// energy component is therefore taken as sign(E) sqrt(m^2 + |p|^2), formed
// in T from the given three-momentum.  (A massless leg nearly collinear with
// a beam makes |M|^2 so sensitive to the off-shellness E - |p| of the input
// that two exact evaluations which read E differently disagree far above
// double rounding; with the projection the result is a function of the
// three-momenta alone.)
template <class T> void load_event(int proc, double mt, const double* mom, int npar, T (*p)[4]) {
  for (int i = 0; i < npar; ++i) {
    for (int m = 1; m < 4; ++m) p[i][m] = T(mom[i * 4 + m]);
    const T mass = T(leg_mass(proc, i, mt));
    const T e = std::sqrt(mass * mass + p[i][1] * p[i][1] + p[i][2] * p[i][2] + p[i][3] * p[i][3]);
    p[i][0] = mom[i * 4] < 0 ? -e : e;
  }
}

// Colour-summed |M_h|^2 for one helicity.
template <class T>
T me_hel(int proc, const Couplings<T>& c, const T (*p)[4], int hel, const std::vector<long double>* C,
         std::vector<cx<T>>& A) {
  if (proc == 0) return std::norm(amp_eemumu(c, p, hel));
  if (is_qq(proc)) return T(qq_colour_factor()) * std::norm(amp_qqtt(c, p, hel, proc == 5 ? 0 : 1, proc == 5 ? 1 : 0));
  if (is_qqg(proc)) return qqg_me_hel(c, p, proc, hel, false);
  int ng = ngluon_of(proc);
  QcdEvent<T> ev = qcd_setup(c, p, ng, hel, -1);
  partial_amps(c, ev, A.data());
  const int nf = int(A.size());
  T sum = 0;
  for (int s = 0; s < nf; ++s) {
    cx<T> row = 0;
    for (int t = 0; t < nf; ++t) row += T((*C)[size_t(s) * nf + t]) * A[t];
    sum += (std::conj(A[s]) * row).real();
  }
  return sum;
}

template <class T>
void run_me(int proc, const oracle_params* prm, const double* mom, int64_t nevt, double* out,
            double* out_hel, int nthreads) {
  const int npar = npar_of(proc);
  const int nhel = 1 << npar;
  const Couplings<T> c(*prm);
  const bool qcd_gluons = proc >= 1 && proc <= 4;
  const std::vector<long double>* C = qcd_gluons ? &colour_matrix_cached(ngluon_of(proc)) : nullptr;
  const int nf = qcd_gluons ? int(factorial(ngluon_of(proc))) : 1;
  const T iden = T(iden_of(proc));
#ifdef _OPENMP
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
  for (int64_t e = 0; e < nevt; ++e) {
    T p[7][4];
    load_event(proc, prm->mt, mom + size_t(e) * npar * 4, npar, p);
    std::vector<cx<T>> A(nf);
    T tot = 0;
    for (int h = 0; h < nhel; ++h) {
      T v = me_hel(proc, c, p, h, C, A);
      if (out_hel) out_hel[size_t(e) * nhel + h] = double(v);
      tot += v;
    }
    if (out) out[e] = double(tot / iden);
  }
}

// ------------------------------------------------------ phase-space points
// Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), written from its
// definition: ten rounds of a multiply-xor network on a 128-bit counter with
// a 64-bit key bumped by the golden-ratio Weyl constants between rounds.
struct Ctr { uint32_t v[4]; };
Ctr philox(Ctr c, uint32_t k0, uint32_t k1) {
  const uint64_t M0 = 0xD2511F53ull, M1 = 0xCD9E8D57ull;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = M0 * c.v[0], p1 = M1 * c.v[2];
    Ctr d;
    d.v[0] = uint32_t(p1 >> 32) ^ c.v[1] ^ k0;
    d.v[1] = uint32_t(p1);
    d.v[2] = uint32_t(p0 >> 32) ^ c.v[3] ^ k1;
    d.v[3] = uint32_t(p0);
    c = d;
  }
  return c;
}
// 53-bit uniform in [0, 1) from two 32-bit words
double unit53(uint32_t a, uint32_t b) {
  return double((uint64_t(a >> 5) << 26) | uint64_t(b >> 6)) / 9007199254740992.0;
}
// the four uniforms (cos theta, phi, energy factors) of final particle i of event e
void event_uniforms(int64_t e, int i, uint64_t seed, double* u) {
  const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
  for (int half = 0; half < 2; ++half) {
    Ctr c{{uint32_t(e), uint32_t(uint64_t(e) >> 32), uint32_t(2 * i + half), 0u}};
    Ctr r = philox(c, k0, k1);
    u[2 * half] = unit53(r.v[0], r.v[1]);
    u[2 * half + 1] = unit53(r.v[2], r.v[3]);
  }
}

// RAMBO (Kleiss, Stirling, Ellis 1986) for one event, in double, with the
// massless invariant mass as sum_{i<j} q0_i q0_j |n_i - n_j|^2, a two-body
// final state rebuilt back to back along RAMBO's direction, and Newton's
// method for massive final states.
void rambo_event(int64_t e, int n, const double* mass, double sqrt_s, uint64_t seed, double* out) {
  const double pi = std::acos(-1.0);
  std::vector<double> q0(n), nh(3 * n), p(4 * n);
  for (int i = 0; i < n; ++i) {
    double u[4];
    event_uniforms(e, i, seed, u);
    const double c = 2 * u[0] - 1, phi = 2 * pi * u[1];
    q0[i] = -std::log((1 - u[2]) * (1 - u[3]));
    const double st = std::sqrt(std::max(0.0, 1 - c * c));
    nh[3 * i] = st * std::cos(phi);
    nh[3 * i + 1] = st * std::sin(phi);
    nh[3 * i + 2] = c;
  }
  double Q[4] = {0, 0, 0, 0}, M2 = 0;
  for (int i = 0; i < n; ++i) {
    Q[0] += q0[i];
    for (int k = 0; k < 3; ++k) Q[k + 1] += q0[i] * nh[3 * i + k];
    for (int j = i + 1; j < n; ++j) {
      double d2 = 0;
      for (int k = 0; k < 3; ++k) d2 += (nh[3 * i + k] - nh[3 * j + k]) * (nh[3 * i + k] - nh[3 * j + k]);
      M2 += q0[i] * q0[j] * d2;
    }
  }
  const double M = std::sqrt(M2), gam = Q[0] / M, a = 1 / (1 + gam), x = sqrt_s / M;
  const double b[3] = {-Q[1] / M, -Q[2] / M, -Q[3] / M};
  for (int i = 0; i < n; ++i) {
    double qv[3], bq = 0;
    for (int k = 0; k < 3; ++k) { qv[k] = q0[i] * nh[3 * i + k]; bq += b[k] * qv[k]; }
    p[4 * i] = x * (gam * q0[i] + bq);
    for (int k = 0; k < 3; ++k) p[4 * i + 1 + k] = x * (qv[k] + b[k] * q0[i] + a * bq * b[k]);
  }
  if (n == 2) {
    const double pn = std::sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
    const double e1 = (sqrt_s * sqrt_s + mass[0] * mass[0] - mass[1] * mass[1]) / (2 * sqrt_s);
    const double pa = std::sqrt(std::max(0.0, e1 * e1 - mass[0] * mass[0]));
    double dir[3] = {p[1] / pn, p[2] / pn, p[3] / pn};
    p[0] = e1;
    p[4] = sqrt_s - e1;
    for (int k = 0; k < 3; ++k) { p[1 + k] = pa * dir[k]; p[5 + k] = -pa * dir[k]; }
  } else {
    double msum = 0;
    for (int i = 0; i < n; ++i) msum += mass[i];
    if (msum > 0) {
      double xi = std::sqrt(1 - (msum / sqrt_s) * (msum / sqrt_s));
      for (int it = 0; it < 30; ++it) {
        double f = -sqrt_s, df = 0;
        for (int i = 0; i < n; ++i) {
          const double en = std::sqrt(mass[i] * mass[i] + xi * xi * p[4 * i] * p[4 * i]);
          f += en;
          df += xi * p[4 * i] * p[4 * i] / en;
        }
        if (std::fabs(f) <= 4e-16 * sqrt_s) break;
        xi -= f / df;
      }
      for (int i = 0; i < n; ++i) {
        p[4 * i] = std::sqrt(mass[i] * mass[i] + xi * xi * p[4 * i] * p[4 * i]);
        for (int k = 1; k < 4; ++k) p[4 * i + k] *= xi;
      }
    }
  }
  const double h = sqrt_s / 2;
  const double beams[8] = {h, 0, 0, h, h, 0, 0, -h};
  std::memcpy(out, beams, sizeof(beams));
  std::memcpy(out + 8, p.data(), sizeof(double) * 4 * n);
}

// ----------------------------------------------- importance-sampled points
// Sequential two-body splitting (the structure of madevent's phase-space
// channels): the centre-of-mass system splits off the last final particle
// and a remainder, the remainder the next-to-last, ..., and the last
// remainder decays into final particles 1 and 2.  Per split k the uniforms
// are Philox words (event, 0x10000 + 2k + half): u0 the remainder's mass,
// u1 the polar angle, u2 the azimuth, all in the decaying system's rest
// frame (reached by a pure boost) with the polar axis along z.
//   remainder mass: M^2 = Mmin^2 + (1 - u0^2)(Mmax^2 - Mmin^2), favouring a
//     soft splitting (M near its maximum); dM^2/du0 = 2 u0 (Mmax^2 - Mmin^2);
//     the distances to both ends of the range are carried exactly (no
//     cancellation in the two-body momenta near a threshold, 1 - u0^2 taken
//     as (1 - u0)(1 + u0))
//   polar angle: c = sqrt(1+eps) tanh(y), y uniform in [-Y, Y] with
//     Y = atanh(1/sqrt(1+eps)), eps = 1/100, so that c covers [-1, 1] with a
//     density ~ 1/(1 + eps - c^2) peaked along the beams;
//     dc/du1 = 2Y (1 + eps - c^2)/sqrt(1+eps) = 2Y sqrt(1+eps)/cosh^2(y)
//   azimuth: phi = 2 pi u2.
// Weight (phase-space Jacobian for dPhi_n = (2pi)^4 delta^4 prod d^3p /
// ((2pi)^3 2E)), from the factorisation dPhi_n = prod_k dPhi_2(k) prod
// dM_k^2/(2pi) with dPhi_2 = |p*|/(16 pi^2 M) dcos dphi:
//   W = prod_splits |p*|/(16 pi^2 M) (dc/du1)(2 pi) x prod_masses 2 u0 (Mmax^2 - Mmin^2)/(2 pi).
void boost_to_lab(const double* P, double M, double* p) {
  // p: four-momentum in the rest frame of P (mass M) -> lab
  const double e = (P[0] * p[0] + P[1] * p[1] + P[2] * p[2] + P[3] * p[3]) / M;
  const double f = (p[0] + e) / (P[0] + M);
  p[0] = e;
  for (int k = 1; k < 4; ++k) p[k] += f * P[k];
}

void sample_event(int64_t e, int n, const double* mass, double sqrt_s, uint64_t seed, double* out, double* w) {
  const double pi = std::acos(-1.0), eps = 0.01;
  const double se = std::sqrt(1 + eps), Y = std::atanh(1 / se);
  const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
  std::vector<double> p(4 * n);
  double P[4] = {sqrt_s, 0, 0, 0}, M = sqrt_s, W = 1.0;
  double mrest = 0;
  for (int i = 0; i < n; ++i) mrest += mass[i];
  double gap = sqrt_s - mrest;                  // M minus the sum of the masses it still holds
  // particles split off in the order n-1, n-2, ..., 2, then (0, 1) together
  for (int k = 0; k < n - 1; ++k) {
    double u[4];
    for (int half = 0; half < 2; ++half) {
      Ctr c{{uint32_t(e), uint32_t(uint64_t(e) >> 32), uint32_t(0x10000 + 2 * k + half), 0u}};
      Ctr r = philox(c, k0, k1);
      u[2 * half] = unit53(r.v[0], r.v[1]);
      u[2 * half + 1] = unit53(r.v[2], r.v[3]);
    }
    const bool last = k == n - 2;
    const int ja = last ? 1 : n - 1 - k;        // the particle split off (the t~ at the last split)
    const double ma = mass[ja];
    mrest -= ma;
    double Mr, thr;                             // remainder mass; M - ma - Mr
    if (last) {
      Mr = mass[0];
      thr = gap;
    } else {
      // hi^2 - lo^2 = gap (hi + lo) and hi - Mr = u0^2 (hi^2 - lo^2) / (hi + Mr):
      // no cancellation near either end of the range
      const double lo = mrest, hi = M - ma, d2 = gap * (hi + lo);
      const double x = (1 - u[0]) * (1 + u[0]);
      Mr = std::sqrt(lo * lo + x * d2);
      thr = u[0] * u[0] * d2 / (hi + Mr);
      gap = x * d2 / (Mr + lo);
      W *= 2 * u[0] * d2 / (2 * pi);
    }
    const double lam = std::sqrt(std::max(0.0, thr * (M + ma + Mr) * (M - ma + Mr) * (M + ma - Mr)));
    const double ps = lam / (2 * M);
    const double y = (2 * u[1] - 1) * Y;
    const double c = se * std::tanh(y), ch = std::cosh(y);
    const double st = std::sqrt(std::max(0.0, 1 - c * c)), phi = 2 * pi * u[2];
    // dc/du1 = 2Y (1 + eps - c^2)/sqrt(1+eps) = 2Y sqrt(1+eps)/cosh^2(y)
    W *= ps / (16 * pi * pi * M) * (2 * Y * se / (ch * ch)) * (2 * pi);
    double pa[4] = {std::sqrt(ma * ma + ps * ps), ps * st * std::cos(phi), ps * st * std::sin(phi), ps * c};
    double pr[4] = {std::sqrt(Mr * Mr + ps * ps), -pa[1], -pa[2], -pa[3]};
    boost_to_lab(P, M, pa);
    boost_to_lab(P, M, pr);
    for (int q = 0; q < 4; ++q) p[4 * ja + q] = pa[q];
    if (last) {
      for (int q = 0; q < 4; ++q) p[q] = pr[q];
    } else {
      for (int q = 0; q < 4; ++q) P[q] = pr[q];
      M = Mr;
    }
  }
  const double h = sqrt_s / 2;
  const double beams[8] = {h, 0, 0, h, h, 0, 0, -h};
  std::memcpy(out, beams, sizeof(beams));
  std::memcpy(out + 8, p.data(), sizeof(double) * 4 * n);
  *w = W;
}

}  // namespace

extern "C" {

int oracle_sample(int64_t nevt, int nfinal, const double* masses, double sqrt_s, uint64_t seed, double* out,
                  double* weight) {
  if (nevt < 0 || nfinal < 2 || nfinal > 5 || !masses || (nevt > 0 && (!out || !weight))) return -1;
  double msum = 0;
  for (int i = 0; i < nfinal; ++i) msum += masses[i];
  if (!(msum < sqrt_s)) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < nevt; ++e)
    sample_event(e, nfinal, masses, sqrt_s, seed, out + e * 4 * (nfinal + 2), weight + e);
  return 0;
}

int oracle_uniforms(int64_t nevt, int nfinal, uint64_t seed, double* out) {
  if (nevt < 0 || nfinal < 1 || (nevt > 0 && !out)) return -1;
  for (int64_t e = 0; e < nevt; ++e)
    for (int i = 0; i < nfinal; ++i) event_uniforms(e, i, seed, out + (e * nfinal + i) * 4);
  return 0;
}

int oracle_rambo(int64_t nevt, int nfinal, const double* masses, double sqrt_s, uint64_t seed, double* out) {
  if (nevt < 0 || nfinal < 2 || nfinal > 5 || !masses || (nevt > 0 && !out)) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < nevt; ++e) rambo_event(e, nfinal, masses, sqrt_s, seed, out + e * 4 * (nfinal + 2));
  return 0;
}


int oracle_npar(int proc) { return npar_of(proc); }
int oracle_ncolor(int proc) {
  if (is_qqg(proc)) return 5;   // diagram basis
  return proc == 0 || is_qq(proc) ? 1 : (npar_of(proc) < 0 ? -1 : int(factorial(ngluon_of(proc))));
}

int oracle_me_gauge(int proc, const oracle_params* p, const double* mom, int64_t nevt, double* out) {
  if (!is_qqg(proc) || !p || nevt < 0 || (nevt > 0 && (!mom || !out))) return -1;
  const Couplings<double> c(*p);
  for (int64_t e = 0; e < nevt; ++e) {
    double pp[7][4];
    load_event(proc, p->mt, mom + size_t(e) * 5 * 4, 5, pp);
    double tot = 0;
    for (int h = 0; h < 32; ++h) tot += qqg_me_hel(c, pp, proc, h, true);
    out[e] = tot / iden_of(proc);
  }
  return 0;
}
double oracle_iden(int proc) { return npar_of(proc) < 0 ? -1.0 : iden_of(proc); }

int oracle_me(int proc, const oracle_params* p, const double* mom, int64_t nevt, double* out,
              int use_long_double, int nthreads) {
  if (npar_of(proc) < 0 || !p || nevt < 0 || (nevt > 0 && (!mom || !out))) return -1;
  if (use_long_double) run_me<long double>(proc, p, mom, nevt, out, nullptr, nthreads);
  else run_me<double>(proc, p, mom, nevt, out, nullptr, nthreads);
  return 0;
}

int oracle_me_hel(int proc, const oracle_params* p, const double* mom, int64_t nevt, double* out,
                  int nthreads) {
  if (npar_of(proc) < 0 || !p || nevt < 0 || (nevt > 0 && (!mom || !out))) return -1;
  run_me<double>(proc, p, mom, nevt, nullptr, out, nthreads);
  return 0;
}

int oracle_partial_amps(int proc, const oracle_params* prm, const double* mom, int hel,
                        int gauge_leg, double* out) {
  const int npar = npar_of(proc);
  if (npar < 0 || !prm || !mom || !out || hel < 0 || hel >= (1 << npar)) return -1;
  const Couplings<double> c(*prm);
  double p[7][4];
  load_event(proc, prm->mt, mom, npar, p);
  if (is_qqg(proc)) return -1;
  if (proc == 0 || is_qq(proc)) {
    if (gauge_leg >= 0) return -1;
    std::complex<double> a = proc == 0 ? amp_eemumu(c, p, hel)
                                       : amp_qqtt(c, p, hel, proc == 5 ? 0 : 1, proc == 5 ? 1 : 0);
    out[0] = a.real(); out[1] = a.imag();
    return 0;
  }
  if (gauge_leg >= 0 && (gauge_leg == 2 || gauge_leg == 3 || gauge_leg >= npar)) return -1;
  int ng = ngluon_of(proc);
  QcdEvent<double> ev = qcd_setup(c, p, ng, hel, gauge_leg);
  std::vector<std::complex<double>> A(factorial(ng));
  partial_amps(c, ev, A.data());
  for (size_t i = 0; i < A.size(); ++i) { out[2 * i] = A[i].real(); out[2 * i + 1] = A[i].imag(); }
  return 0;
}

int oracle_dressed_amp(int proc, const oracle_params* prm, const double* mom, int hel,
                       const int* colours, double* out) {
  const int npar = npar_of(proc);
  if (proc < 1 || proc > 4 || npar < 0 || !prm || !mom || !colours || !out || hel < 0 || hel >= (1 << npar))
    return -1;
  int ng = ngluon_of(proc);
  for (int g = 0; g < ng; ++g)
    if (colours[g] < 0 || colours[g] > 7) return -1;
  if (colours[ng] < 0 || colours[ng] > 2 || colours[ng + 1] < 0 || colours[ng + 1] > 2) return -1;
  const Couplings<double> c(*prm);
  double p[7][4];
  load_event(proc, prm->mt, mom, npar, p);
  QcdEvent<double> ev = qcd_setup(c, p, ng, hel, -1);
  std::complex<double> a = dressed_amp(c, ev, colours);
  out[0] = a.real(); out[1] = a.imag();
  return 0;
}

int oracle_colour_basis(int ngluons, const int* colours, double* out) {
  if (ngluons < 1 || ngluons > 5 || !colours || !out) return -1;
  std::vector<std::complex<double>> v(factorial(ngluons));
  colour_basis_values(ngluons, colours, v.data());
  for (size_t i = 0; i < v.size(); ++i) { out[2 * i] = v[i].real(); out[2 * i + 1] = v[i].imag(); }
  return 0;
}

int oracle_colour_matrix(int ngluons, double* out) {
  if (ngluons < 1 || ngluons > 5 || !out) return -1;
  const std::vector<long double>& C = colour_matrix_cached(ngluons);
  for (size_t q = 0; q < C.size(); ++q) out[q] = double(C[q]);
  return 0;
}

}  // extern "C"
