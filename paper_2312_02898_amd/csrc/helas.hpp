// Device-side helicity-amplitude building blocks for gfx950 (one event per lane).
//
// HELAS-style functions (Murayama, Watanabe, Hagiwara, KEK-91-11) written from
// the Feynman rules in the chiral (Weyl) representation:
//   gamma^mu = [[0, sigma^mu], [sigmabar^mu, 0]], sigma = (1, s_k),
//   sigmabar = (1, -s_k), gamma^5 = diag(-1, 1); components 0,1 are
//   left-handed, 2,3 right-handed.
// Every fermion-vector vertex is  i gamma^mu (gL P_L + gR P_R)  with real gL, gR:
//   QCD  q qbar g : gL = gR = g_s            (rule +i g_s gamma^mu t^a)
//   QED  f fbar a : gL = gR = -e Q
//   Z    f fbar Z : gL = -e cL, gR = -e cR
// Propagators: fermion i(P/+m)/(P^2-m^2+i m Gamma); gluon/photon -i g/K^2;
// Z -i(g - K K/M^2)/(K^2-M^2+i M Gamma).  The three-gluon vertex is
// g f^{abc} V^{mu nu rho}(k,p,q), the four-gluon vertex -i g^2 (f f)(g g - g g);
// colour factors are handled outside these functions.
//
// Wavefunctions: column spinors (u for incoming fermions, v for outgoing
// antifermions), row spinors (ubar for outgoing fermions, vbar for incoming
// antifermions; stored so that rowspinor.col = sum_i r_i c_i) and vectors
// with upper Lorentz index.  Momenta K are the momentum that the current
// carries into the vertex it feeds; P along the fermion-number arrow.
//
// T is the arithmetic type of the wavefunction algebra (double for the FP64
// form, float for the mixed form).  Momenta, p^2 and propagator denominators
// are always formed in double by the caller and rounded to T there.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

template <class T> struct cx { T r, i; };

template <class T> __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <class T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <class T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <class T> __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.r, -a.i}; }
template <class T> __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <class T> __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.r, s * a.i}; }
template <class T> __device__ __forceinline__ cx<T> operator*(cx<T> a, T s) { return {s * a.r, s * a.i}; }
template <class T> __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.i, a.r}; }      // i a
template <class T> __device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.i, -a.r}; }     // -i a
template <class T> __device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.r, -a.i}; }
// a*b + c
template <class T> __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
  return {a.r * b.r - a.i * b.i + c.r, a.r * b.i + a.i * b.r + c.i};
}

template <class T> struct wf {                   // spinor or vector wavefunction
  using value_type = T;
  cx<T> c[4];
};
template <class T> struct mom { T k[4]; };      // real momentum in arithmetic type T

// ------------------------------------------------ structurally known zeros
// An external massless vector has a zero time component and a real z
// component in the helicity basis used here (ext_eps).  Strict IEEE
// arithmetic may not drop x*0 or x+0 (x could be NaN or infinite, the zero
// negative), so these components are carried as types instead: zero_t is an
// exact 0, re<T> a complex number whose imaginary part is exactly 0.  The
// vector vertices below read their vector operands through comp<M>(), so the
// terms such a component removes are never evaluated.
struct zero_t {};
template <class T> struct re { T r; };

template <class T> struct epsw {                 // external massless vector (0, c1, c2, c3 real)
  using value_type = T;
  cx<T> c1, c2;
  T c3;
};

template <int M, class T> __device__ __forceinline__ cx<T> comp(const wf<T>& w) { return w.c[M]; }
template <int M, class T> __device__ __forceinline__ auto comp(const epsw<T>& w) {
  if constexpr (M == 0) return zero_t{};
  else if constexpr (M == 1) return w.c1;
  else if constexpr (M == 2) return w.c2;
  else return re<T>{w.c3};
}

__device__ __forceinline__ zero_t operator*(zero_t, zero_t) { return {}; }
template <class X> __device__ __forceinline__ zero_t operator*(zero_t, const X&) { return {}; }
template <class X> __device__ __forceinline__ zero_t operator*(const X&, zero_t) { return {}; }
__device__ __forceinline__ zero_t operator+(zero_t, zero_t) { return {}; }
template <class X> __device__ __forceinline__ X operator+(zero_t, const X& x) { return x; }
template <class X> __device__ __forceinline__ X operator+(const X& x, zero_t) { return x; }
__device__ __forceinline__ zero_t operator-(zero_t, zero_t) { return {}; }
template <class X> __device__ __forceinline__ X operator-(zero_t, const X& x) { return -x; }
template <class X> __device__ __forceinline__ X operator-(const X& x, zero_t) { return x; }
__device__ __forceinline__ zero_t operator-(zero_t) { return {}; }
__device__ __forceinline__ zero_t mul_i(zero_t) { return {}; }
__device__ __forceinline__ zero_t mul_mi(zero_t) { return {}; }

template <class T> __device__ __forceinline__ re<T> operator-(re<T> a) { return {-a.r}; }
template <class T> __device__ __forceinline__ re<T> operator+(re<T> a, re<T> b) { return {a.r + b.r}; }
template <class T> __device__ __forceinline__ re<T> operator-(re<T> a, re<T> b) { return {a.r - b.r}; }
template <class T> __device__ __forceinline__ re<T> operator*(re<T> a, re<T> b) { return {a.r * b.r}; }
template <class T> __device__ __forceinline__ re<T> operator*(T s, re<T> a) { return {s * a.r}; }
template <class T> __device__ __forceinline__ re<T> operator*(re<T> a, T s) { return {a.r * s}; }
template <class T> __device__ __forceinline__ cx<T> operator*(re<T> a, cx<T> b) { return {a.r * b.r, a.r * b.i}; }
template <class T> __device__ __forceinline__ cx<T> operator*(cx<T> b, re<T> a) { return {b.r * a.r, b.i * a.r}; }
template <class T> __device__ __forceinline__ cx<T> operator+(re<T> a, cx<T> b) { return {a.r + b.r, b.i}; }
template <class T> __device__ __forceinline__ cx<T> operator+(cx<T> b, re<T> a) { return {b.r + a.r, b.i}; }
template <class T> __device__ __forceinline__ cx<T> operator-(re<T> a, cx<T> b) { return {a.r - b.r, -b.i}; }
template <class T> __device__ __forceinline__ cx<T> operator-(cx<T> b, re<T> a) { return {b.r - a.r, b.i}; }

// Widening to a full complex number.
template <class T> __device__ __forceinline__ cx<T> as_cx(cx<T> x) { return x; }
template <class T> __device__ __forceinline__ cx<T> as_cx(re<T> x) { return {x.r, T(0)}; }
template <class T> __device__ __forceinline__ cx<T> as_cx(zero_t) { return {T(0), T(0)}; }

template <class T> __device__ __forceinline__ mom<T> to_mom(const double* K) {
  return mom<T>{{T(K[0]), T(K[1]), T(K[2]), T(K[3])}};
}
__device__ __forceinline__ double msq(const double* K) {
  return K[0] * K[0] - K[1] * K[1] - K[2] * K[2] - K[3] * K[3];
}
// K^2 from light-cone components along the beam axis: K+ = K0 + K3,
// K- = K0 - K3.
__device__ __forceinline__ double msq_lc(double kp, double km, double kx, double ky) {
  return kp * km - kx * kx - ky * ky;
}
// Light-cone components E + pz and E - pz of an on-shell momentum of mass m
// (m^2 passed), each without cancellation: the small one of the two is
// (m^2 + pT^2) divided by the large one.
__device__ __forceinline__ double lc_plus(const double* p, double m2) {
  return p[3] >= 0 ? p[0] + p[3] : (m2 + p[1] * p[1] + p[2] * p[2]) / (p[0] - p[3]);
}
__device__ __forceinline__ double lc_minus(const double* p, double m2) {
  return p[3] <= 0 ? p[0] - p[3] : (m2 + p[1] * p[1] + p[2] * p[2]) / (p[0] + p[3]);
}
// The small one of E +- pz, (m^2 + pT^2) / (E + |pz|), and the light-cone
// components from it (s: the small component, from a per-event cache).
__device__ __forceinline__ double lc_small(const double* p, double m2) {
  return (m2 + p[1] * p[1] + p[2] * p[2]) / (p[0] + fabs(p[3]));
}
__device__ __forceinline__ double lc_plus_s(const double* p, double s) { return p[3] >= 0 ? p[0] + p[3] : s; }
__device__ __forceinline__ double lc_minus_s(const double* p, double s) { return p[3] <= 0 ? p[0] - p[3] : s; }
// (a + b)^2 = 2 a.b for two massless on-shell momenta, as
// |E_b a_vec - E_a b_vec|^2 / (E_a E_b): the difference vector is small when
// the two are nearly collinear and is formed with one rounding per component,
// where E_a E_b - a_vec.b_vec would cancel.
__device__ __forceinline__ double msq_pair0(const double* a, const double* b) {
  const double wx = fma(b[0], a[1], -(a[0] * b[1]));
  const double wy = fma(b[0], a[2], -(a[0] * b[2]));
  const double wz = fma(b[0], a[3], -(a[0] * b[3]));
  return (wx * wx + wy * wy + wz * wz) / (a[0] * b[0]);
}
// External momenta on the mass shell.  The energy component of each leg is
// recomputed as sqrt(m^2 + |p|^2) (with the sign of the given one): a double
// input is on shell only to rounding, and near collinear configurations the
// result is sensitive to that rounding.  MASSIVE: bit i set if leg i has
// mass mt.
template <unsigned MASSIVE, int N>
__device__ __forceinline__ void load_on_shell(const double* mom, double (&p)[N][4], double mt) {
  const double2* src = reinterpret_cast<const double2*>(mom);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double2 a = src[2 * i], b = src[2 * i + 1];
    const double m2 = (MASSIVE >> i & 1u) ? mt * mt : 0.0;
    p[i][1] = a.y; p[i][2] = b.x; p[i][3] = b.y;
    p[i][0] = copysign(sqrt(m2 + a.y * a.y + b.x * b.x + b.y * b.y), a.x);
  }
}

// Minkowski product of complex 4-vectors (no conjugation).
// Either operand may be a wf or an epsw.
template <class A, class B> __device__ __forceinline__ cx<typename A::value_type> dot(const A& a, const B& b) {
  using T = typename A::value_type;
  return as_cx<T>(((comp<0>(a) * comp<0>(b) - comp<1>(a) * comp<1>(b)) - comp<2>(a) * comp<2>(b)) -
                  comp<3>(a) * comp<3>(b));
}
// Minkowski product of a real momentum with a complex vector.
template <class T, class W> __device__ __forceinline__ cx<T> dot(const mom<T>& k, const W& b) {
  return as_cx<T>(((k.k[0] * comp<0>(b) - k.k[1] * comp<1>(b)) - k.k[2] * comp<2>(b)) - k.k[3] * comp<3>(b));
}

// ------------------------------------------------------- external states
// Two-component helicity eigenstates chi_+/- of sigma.p_hat, computed in FP64.
// |p|+p_z is formed as p_T^2/(|p|-p_z) for p_z < 0 to avoid cancellation; on
// the negative z axis chi_+ = (0,1), chi_- = (-1,0).
struct chi2 { double ar, ai, br, bi; };
__device__ __forceinline__ void helicity_chis(const double* p, chi2& cp, chi2& cm) {
  const double pt2 = p[1] * p[1] + p[2] * p[2];
  const double pp = sqrt(pt2 + p[3] * p[3]);
  const double a = p[3] >= 0 ? pp + p[3] : (pt2 > 0 ? pt2 / (pp - p[3]) : 0.0);
  if (a > 0) {
    const double n = 1.0 / sqrt(2.0 * pp * a);
    cp = chi2{a * n, 0.0, p[1] * n, p[2] * n};
    cm = chi2{-p[1] * n, p[2] * n, a * n, 0.0};
  } else {
    cp = chi2{0.0, 0.0, 1.0, 0.0};
    cm = chi2{-1.0, 0.0, 0.0, 0.0};
  }
}
// sqrt(E -+ |p|), sqrt(E + |p|): omega_- is taken as m/omega_+ (exactly 0 when massless).
__device__ __forceinline__ void omegas(const double* p, double m, double& wp, double& wm) {
  const double pp = sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
  wp = sqrt(p[0] + pp);
  wm = m == 0.0 ? 0.0 : m / wp;
}
template <class T> __device__ __forceinline__ cx<T> c2(double r, double i) { return cx<T>{T(r), T(i)}; }

// u(p,lam) = (omega_{-lam} chi_lam ; omega_lam chi_lam)   (column)
template <class T> __device__ __forceinline__ wf<T> ext_u(const double* p, double m, int lam) {
  chi2 cp, cm; helicity_chis(p, cp, cm);
  double wp, wm; omegas(p, m, wp, wm);
  const chi2 x = lam > 0 ? cp : cm;
  const double lo = lam > 0 ? wm : wp, hi = lam > 0 ? wp : wm;
  wf<T> w;
  w.c[0] = c2<T>(lo * x.ar, lo * x.ai); w.c[1] = c2<T>(lo * x.br, lo * x.bi);
  w.c[2] = c2<T>(hi * x.ar, hi * x.ai); w.c[3] = c2<T>(hi * x.br, hi * x.bi);
  return w;
}
// v(p,lam) = (-lam omega_lam chi_{-lam} ; lam omega_{-lam} chi_{-lam})   (column)
template <class T> __device__ __forceinline__ wf<T> ext_v(const double* p, double m, int lam) {
  chi2 cp, cm; helicity_chis(p, cp, cm);
  double wp, wm; omegas(p, m, wp, wm);
  const chi2 x = lam > 0 ? cm : cp;
  const double up = lam > 0 ? -wp : wm;         // -lam omega_lam
  const double dn = lam > 0 ? wm : -wp;         // lam omega_{-lam}
  wf<T> w;
  w.c[0] = c2<T>(up * x.ar, up * x.ai); w.c[1] = c2<T>(up * x.br, up * x.bi);
  w.c[2] = c2<T>(dn * x.ar, dn * x.ai); w.c[3] = c2<T>(dn * x.br, dn * x.bi);
  return w;
}
// Dirac adjoint psi^dagger gamma^0 as a row: (conj psi_R, conj psi_L).
template <class T> __device__ __forceinline__ wf<T> bar(const wf<T>& s) {
  wf<T> r;
  r.c[0] = cconj(s.c[2]); r.c[1] = cconj(s.c[3]);
  r.c[2] = cconj(s.c[0]); r.c[3] = cconj(s.c[1]);
  return r;
}
// Massless vector polarisation eps(k,lam) = (-lam e1 - i e2)/sqrt2,
// e1 = (0, cos th cos ph, cos th sin ph, -sin th), e2 = (0, -sin ph, cos ph, 0);
// phi = 0 on the z axis.  conj_out selects eps* (outgoing vectors).
// The helicity enters only as a sign: with a = (cth cph, cth sph, sth)/sqrt2
// and b = (sph, -cph)/sqrt2 (eps_base), eps = (0, -lam a0 + i s b0,
// -lam a1 + i s b1, lam a2) with s = -1 for eps*, +1 otherwise.
struct EpsBase { double a0, a1, a2, b0, b1; };
__device__ __forceinline__ EpsBase eps_base(const double* k) {
  const double pt2 = k[1] * k[1] + k[2] * k[2];
  const double pt = sqrt(pt2);
  const double kk = sqrt(pt2 + k[3] * k[3]);
  double cph = 1.0, sph = 0.0, cth, sth;
  if (pt > 0) { cph = k[1] / pt; sph = k[2] / pt; cth = k[3] / kk; sth = pt / kk; }
  else { cth = k[3] >= 0 ? 1.0 : -1.0; sth = 0.0; }
  const double r2 = 0.70710678118654752440;
  return EpsBase{cth * cph * r2, cth * sph * r2, sth * r2, sph * r2, -cph * r2};
}
// eps from its base values (already rounded to T): only sign changes.
template <class T> __device__ __forceinline__ epsw<T> eps_from_base(T a0, T a1, T a2, T b0, T b1, int lam,
                                                                    bool conj_out) {
  epsw<T> e;
  const T l = T(lam), s = conj_out ? T(-1) : T(1);
  e.c1 = cx<T>{-l * a0, s * b0};
  e.c2 = cx<T>{-l * a1, s * b1};
  e.c3 = l * a2;
  return e;
}
template <class T> __device__ __forceinline__ epsw<T> ext_eps(const double* k, int lam, bool conj_out) {
  const EpsBase b = eps_base(k);
  return eps_from_base<T>(T(b.a0), T(b.a1), T(b.a2), T(b.b0), T(b.b1), lam, conj_out);
}

// --------------------------------------------------- fermion-vector vertex
// Components of J.sigma = [[b, -d], [-c, a]] and J.sigmabar = [[a, d], [c, b]],
// a = J0+J3, b = J0-J3, c = J1 + i J2, d = J1 - i J2.
// For an external vector (epsw) a and b are real.
template <class A, class B, class C, class D> struct jsig { A a; B b; C c; D d; };
template <class W> __device__ __forceinline__ auto sig(const W& J) {
  const auto a = comp<0>(J) + comp<3>(J);
  const auto b = comp<0>(J) - comp<3>(J);
  const auto c = comp<1>(J) + mul_i(comp<2>(J));
  const auto d = comp<1>(J) - mul_i(comp<2>(J));
  return jsig<decltype(a), decltype(b), decltype(c), decltype(d)>{a, b, c, d};
}

// Amplitude  rbar [i gamma.J (gL P_L + gR P_R)] psi.
template <class T, class W>
__device__ __forceinline__ cx<T> ffv_amp(const wf<T>& r, const W& J, const wf<T>& s, T gL, T gR) {
  const auto q = sig(J);
  // r_L (J.sigma) psi_R
  cx<T> x = r.c[0] * (q.b * s.c[2] - q.d * s.c[3]) + r.c[1] * (q.a * s.c[3] - q.c * s.c[2]);
  // r_R (J.sigmabar) psi_L
  cx<T> y = r.c[2] * (q.a * s.c[0] + q.d * s.c[1]) + r.c[3] * (q.c * s.c[0] + q.b * s.c[1]);
  return mul_i(gR * x + gL * y);
}

// Half contractions, for amplitudes that share a row spinor and a vector
// (or a vector and a column spinor):
//   row  s = rbar gamma.J (gL P_L + gR P_R),   column  x = gamma.J (gL P_L + gR P_R) psi,
// and the amplitude  i (row . column).
template <class T, class W>
__device__ __forceinline__ wf<T> ffv_half_row(const wf<T>& r, const W& J, T gL, T gR) {
  const auto q = sig(J);
  wf<T> o;
  o.c[0] = gL * (r.c[2] * q.a + r.c[3] * q.c);
  o.c[1] = gL * (r.c[2] * q.d + r.c[3] * q.b);
  o.c[2] = gR * (r.c[0] * q.b - r.c[1] * q.c);
  o.c[3] = gR * (r.c[1] * q.a - r.c[0] * q.d);
  return o;
}
template <class T, class W>
__device__ __forceinline__ wf<T> ffv_half_col(const W& J, const wf<T>& s, T gL, T gR) {
  const auto q = sig(J);
  wf<T> o;
  o.c[0] = gR * (q.b * s.c[2] - q.d * s.c[3]);
  o.c[1] = gR * (q.a * s.c[3] - q.c * s.c[2]);
  o.c[2] = gL * (q.a * s.c[0] + q.d * s.c[1]);
  o.c[3] = gL * (q.c * s.c[0] + q.b * s.c[1]);
  return o;
}
template <class T> __device__ __forceinline__ cx<T> amp_dot(const wf<T>& r, const wf<T>& c) {
  cx<T> t = r.c[0] * c.c[0];
  t = cfma(r.c[1], c.c[1], t);
  t = cfma(r.c[2], c.c[2], t);
  t = cfma(r.c[3], c.c[3], t);
  return mul_i(t);
}

// Off-shell column spinor  i(K/+m)/(K^2-m^2+i m G) [i gamma.J (gL P_L+gR P_R)] psi.
// K: momentum along the arrow (into the next vertex); den = 1/(K^2-m^2+i m G).
// m is a T, or zero_t for a massless line; den a cx<T>, or re<T> for a
// massless line (1/K^2).
template <class T, class W, class M, class DN>
__device__ __forceinline__ wf<T> ffv_fin(const wf<T>& s, const W& J, const mom<T>& K, M m, DN den,
                                         T gL, T gR) {
  const auto q = sig(J);
  const cx<T> x0 = gR * (q.b * s.c[2] - q.d * s.c[3]);
  const cx<T> x1 = gR * (q.a * s.c[3] - q.c * s.c[2]);
  const cx<T> x2 = gL * (q.a * s.c[0] + q.d * s.c[1]);
  const cx<T> x3 = gL * (q.c * s.c[0] + q.b * s.c[1]);
  const T kp = K.k[0] + K.k[3], km = K.k[0] - K.k[3];
  const cx<T> kc{K.k[1], K.k[2]}, kd{K.k[1], -K.k[2]};   // K1 + i K2, K1 - i K2
  const auto nd = -den;                                  // i * i * den
  wf<T> o;
  o.c[0] = nd * (km * x2 - kd * x3 + m * x0);
  o.c[1] = nd * (kp * x3 - kc * x2 + m * x1);
  o.c[2] = nd * (kp * x0 + kd * x1 + m * x2);
  o.c[3] = nd * (kc * x0 + km * x1 + m * x3);
  return o;
}

// Off-shell row spinor  rbar [i gamma.J (gL P_L+gR P_R)] i(P/+m)/(P^2-m^2+i m G).
// P: momentum along the arrow (= minus the momentum the row current carries
// into its next vertex).
template <class T, class W, class M, class DN>
__device__ __forceinline__ wf<T> ffv_fout(const wf<T>& r, const W& J, const mom<T>& P, M m, DN den,
                                          T gL, T gR) {
  const auto q = sig(J);
  const cx<T> s0 = gL * (r.c[2] * q.a + r.c[3] * q.c);
  const cx<T> s1 = gL * (r.c[2] * q.d + r.c[3] * q.b);
  const cx<T> s2 = gR * (r.c[0] * q.b - r.c[1] * q.c);
  const cx<T> s3 = gR * (r.c[1] * q.a - r.c[0] * q.d);
  const T kp = P.k[0] + P.k[3], km = P.k[0] - P.k[3];
  const cx<T> kc{P.k[1], P.k[2]}, kd{P.k[1], -P.k[2]};
  const auto nd = -den;
  wf<T> o;
  // (s_L, s_R) [[m, P.sigma], [P.sigmabar, m]]
  o.c[0] = nd * (m * s0 + kp * s2 + kc * s3);
  o.c[1] = nd * (m * s1 + kd * s2 + km * s3);
  o.c[2] = nd * (km * s0 - kc * s1 + m * s2);
  o.c[3] = nd * (kp * s1 - kd * s0 + m * s3);
  return o;
}

// Fermion current  j^mu = rbar gamma^mu (gL P_L + gR P_R) psi  (no factor i).
template <class T>
__device__ __forceinline__ wf<T> ffv_current(const wf<T>& r, const wf<T>& s, T gL, T gR) {
  // r_R sigmabar^mu psi_L
  const cx<T> l0 = r.c[2] * s.c[0] + r.c[3] * s.c[1];
  const cx<T> l1 = -(r.c[2] * s.c[1] + r.c[3] * s.c[0]);
  const cx<T> l2 = mul_i(r.c[2] * s.c[1] - r.c[3] * s.c[0]);
  const cx<T> l3 = r.c[3] * s.c[1] - r.c[2] * s.c[0];
  // r_L sigma^mu psi_R
  const cx<T> h0 = r.c[0] * s.c[2] + r.c[1] * s.c[3];
  const cx<T> h1 = r.c[0] * s.c[3] + r.c[1] * s.c[2];
  const cx<T> h2 = mul_i(r.c[1] * s.c[2] - r.c[0] * s.c[3]);
  const cx<T> h3 = r.c[0] * s.c[2] - r.c[1] * s.c[3];
  wf<T> j;
  j.c[0] = gL * l0 + gR * h0;
  j.c[1] = gL * l1 + gR * h1;
  j.c[2] = gL * l2 + gR * h2;
  j.c[3] = gL * l3 + gR * h3;
  return j;
}
// Off-shell massless vector (gluon, photon): (-i/K^2) (i j^mu) = j^mu / K^2.
template <class T>
__device__ __forceinline__ wf<T> ffv_v0(const wf<T>& r, const wf<T>& s, T inv_k2, T gL, T gR) {
  wf<T> j = ffv_current(r, s, gL, gR);
  for (int m = 0; m < 4; ++m) j.c[m] = inv_k2 * j.c[m];
  return j;
}
// Off-shell massive vector, unitary gauge: den [j^mu - K^mu (K.j)/M^2].
template <class T>
__device__ __forceinline__ wf<T> ffv_vm(const wf<T>& r, const wf<T>& s, const mom<T>& K, T inv_m2, cx<T> den,
                                        T gL, T gR) {
  wf<T> j = ffv_current(r, s, gL, gR);
  const cx<T> kj = dot(K, j) * inv_m2;
  wf<T> o;
  for (int m = 0; m < 4; ++m) o.c[m] = den * (j.c[m] - K.k[m] * kj);
  return o;
}

// ---------------------------------------------------------- gluon vertices
// V^mu(A,B) = A^mu ((k-p).B) + (A.B)(p-q)^mu + B^mu ((q-k).A) with incoming
// momenta p = KA, q = KB and k = -(KA+KB) on the free leg.
template <class T, class WA, class WB>
__device__ __forceinline__ wf<T> vvv_lorentz(const WA& A, const mom<T>& KA, const WB& B, const mom<T>& KB) {
  mom<T> kmp, pmq, qmk;
  for (int m = 0; m < 4; ++m) {
    kmp.k[m] = -T(2) * KA.k[m] - KB.k[m];
    pmq.k[m] = KA.k[m] - KB.k[m];
    qmk.k[m] = T(2) * KB.k[m] + KA.k[m];
  }
  const cx<T> t1 = dot(kmp, B), t2 = dot(A, B), t3 = dot(qmk, A);
  wf<T> v;
  v.c[0] = (comp<0>(A) * t1 + comp<0>(B) * t3) + pmq.k[0] * t2;
  v.c[1] = (comp<1>(A) * t1 + comp<1>(B) * t3) + pmq.k[1] * t2;
  v.c[2] = (comp<2>(A) * t1 + comp<2>(B) * t3) + pmq.k[2] * t2;
  v.c[3] = (comp<3>(A) * t1 + comp<3>(B) * t3) + pmq.k[3] * t2;
  return v;
}
// Off-shell gluon from a three-gluon vertex: (-i/K^2) g V^mu(A,B).
template <class T, class WA, class WB>
__device__ __forceinline__ wf<T> vvv_v(const WA& A, const mom<T>& KA, const WB& B, const mom<T>& KB,
                                       T g_inv_k2) {
  wf<T> v = vvv_lorentz(A, KA, B, KB);
  for (int m = 0; m < 4; ++m) v.c[m] = mul_mi(g_inv_k2 * v.c[m]);
  return v;
}
// Amplitude  g V^{mu nu rho}(k,p,q) X_mu A_nu B_rho with incoming momenta
// k = KX, p = KA, q = KB (KX + KA + KB = 0).
template <class T, class WX, class WA, class WB>
__device__ __forceinline__ cx<T> vvv_amp(const WX& X, const mom<T>& KX, const WA& A, const mom<T>& KA,
                                         const WB& B, const mom<T>& KB, T g) {
  mom<T> kmp, pmq, qmk;
  for (int m = 0; m < 4; ++m) {
    kmp.k[m] = KX.k[m] - KA.k[m];
    pmq.k[m] = KA.k[m] - KB.k[m];
    qmk.k[m] = KB.k[m] - KX.k[m];
  }
  const cx<T> r = dot(X, A) * dot(kmp, B) + dot(A, B) * dot(pmq, X) + dot(B, X) * dot(qmk, A);
  return g * r;
}
// Four-gluon piece for the colour structure f^{x b e} f^{e c d}:
// P^mu(b; c, d) = C^mu (B.D) - D^mu (B.C).
template <class T, class WB, class WC, class WD>
__device__ __forceinline__ wf<T> vvvv_piece(const WB& B, const WC& C, const WD& D) {
  const cx<T> bd = dot(B, D), bc = dot(B, C);
  wf<T> v;
  v.c[0] = as_cx<T>(comp<0>(C) * bd - comp<0>(D) * bc);
  v.c[1] = as_cx<T>(comp<1>(C) * bd - comp<1>(D) * bc);
  v.c[2] = as_cx<T>(comp<2>(C) * bd - comp<2>(D) * bc);
  v.c[3] = as_cx<T>(comp<3>(C) * bd - comp<3>(D) * bc);
  return v;
}
// Identity that the compiler cannot see through: a recomputed wavefunction
// passes one input through it so that it is not merged with the first copy.
template <class T> __device__ __forceinline__ wf<T> opaque(wf<T> w) {
#pragma unroll
  for (int m = 0; m < 4; ++m) asm volatile("" : "+v"(w.c[m].r), "+v"(w.c[m].i));
  return w;
}
template <class T> __device__ __forceinline__ epsw<T> opaque(epsw<T> w) {
  asm volatile("" : "+v"(w.c1.r), "+v"(w.c1.i), "+v"(w.c2.r), "+v"(w.c2.i), "+v"(w.c3));
  return w;
}
__device__ __forceinline__ double opaque_d(double x) {
  asm volatile("" : "+v"(x));
  return x;
}
// Pins a jamp accumulator update where the schedule put it.  Without it the
// optimizer sinks the (pure) additions down to the accumulator's last use,
// which keeps every amplitude alive until then.
template <class T> __device__ __forceinline__ void hold(cx<T>& a) {
  asm volatile("" : "+v"(a.r), "+v"(a.i));
}
template <class T, int N> __device__ __forceinline__ void hold_jamp(cx<T> (&jamp)[N], int k) { hold(jamp[k]); }
// jamps kept in memory are not sunk
template <class J> __device__ __forceinline__ void hold_jamp(J&, int) {}

// Per-event cache of propagator factors: the generated FP32 amplitude
// function reads them from the cache when the kernel passes one (kCached) and
// forms them in place from the momenta otherwise (this type).
struct NoKinCache {
  static constexpr bool kCached = false;
  static constexpr bool kMom = false;
  static constexpr bool kLc = false;   // no light-cone cache either
  __device__ __forceinline__ double lcs(int) const { return 0.0; }
  __device__ __forceinline__ double pair(int) const { return 0.0; }
};

// A momentum copy the compiler cannot identify with the original, for
// recomputed external wavefunctions (which have no wavefunction input).
struct OpaqueMom {
  double v[4];
};
__device__ __forceinline__ OpaqueMom opaque_mom(const double* p) {
  OpaqueMom r;
#pragma unroll
  for (int c = 0; c < 4; ++c) r.v[c] = opaque_d(p[c]);
  return r;
}
template <class T> __device__ __forceinline__ void acc_scaled(wf<T>& o, const wf<T>& v, T s) {
  for (int m = 0; m < 4; ++m) o.c[m] = o.c[m] + s * v.c[m];
}

}  // namespace me
