/*
 * CPU oracle for leading-order squared matrix elements |M|^2.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU path (no headers, helpers, tables or generators).
 *
 * What it computes (the plain definition, paper silent on the formula; the
 * paper, Sec. 2, names the "matrix elements" as the quantity the accelerated
 * code evaluates for each event, Sec. 4 restricts to LO QED/QCD and names the
 * validated processes e+e- -> mu+mu- and gg -> ttbar + 0..3 g):
 *
 *   |M|^2(p) = 1/IDEN * sum_{all helicities} sum_{all colours} |M(p;h,c)|^2
 *
 * with M the sum of all tree-level Feynman diagrams (Peskin-Schroeder Feynman
 * rules, Feynman gauge for gluons/photons, unitary gauge for the Z, fixed
 * widths).  For the QCD processes the oracle evaluates colour-ordered partial
 * amplitudes A(sigma) with a Berends-Giele recursion along the top line and
 * contracts them with the colour matrix C obtained by brute-force SU(3)
 * summation over explicit Gell-Mann matrices.  A second, colour-dressed
 * recursion (literal f^{abc}, t^a with explicit colour indices) is exposed so
 * that the colour-ordered normalisation can be pinned against the literal
 * Lagrangian rules.
 *
 * Conventions shared with callers (interface, not arithmetic):
 *   process ids: 0 "e+ e- > mu+ mu-", 1 "g g > t t~", 2 "g g > t t~ g",
 *                3 "g g > t t~ g g", 4 "g g > t t~ g g g", 5 "u u~ > t t~",
 *                6 "u~ u > t t~" (massless light quark; the q qbar channels
 *                of p p > t t~ beside g g > t t~), 7 "u u~ > t t~ g",
 *                8 "u~ u > t t~ g", 9 "u g > t t~ u", 10 "g u > t t~ u",
 *                11 "u~ g > t t~ u~", 12 "g u~ > t t~ u~" (one jet).
 *   momenta:     double mom[nevt][npar][4], (E,px,py,pz) in GeV, legs 0 and 1
 *                incoming, the others outgoing, leg order = process string.
 *   helicity index h in [0, 2^npar): leg i has helicity +1 if bit i of h is
 *                set, -1 otherwise (physical helicity of the particle).
 *   gluon numbering for colour orderings: gluon legs in increasing leg order
 *                (legs 0,1,4,5,6 -> gluons 0,1,2,3,4); orderings sigma are
 *                enumerated in lexicographic order.
 *
 * Every function returns 0 on success, a negative value on bad arguments.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double alpha_em;     /* fine-structure constant (not running) */
  double sin2w;        /* sin^2 theta_W, taken as an input */
  double mz, wz;       /* Z mass and width (GeV) */
  double mt, wt;       /* top mass and width (GeV) */
  double alpha_s;      /* fixed strong coupling */
  int32_t tchan_zero_width; /* 1: width 0 in t-channel top propagators */
  int32_t reserved;
} oracle_params;

int oracle_npar(int proc);
int oracle_ncolor(int proc);
double oracle_iden(int proc);

/* Helicity- and colour-summed, averaged |M|^2 per event.  use_long_double
 * selects 80-bit extended arithmetic (for rounding adjudication).  nthreads<=0
 * uses the OpenMP default. */
int oracle_me(int proc, const oracle_params* p, const double* mom, int64_t nevt,
              double* out, int use_long_double, int nthreads);

/* Colour-summed (not averaged) |M_h|^2 for every helicity h, out[nevt][2^npar]. */
int oracle_me_hel(int proc, const oracle_params* p, const double* mom, int64_t nevt,
                  double* out, int nthreads);

/* Processes 7..12: as oracle_me with the gluon's polarisation replaced by
 * its momentum k/k^0 (gauge check: must vanish). */
int oracle_me_gauge(int proc, const oracle_params* p, const double* mom, int64_t nevt, double* out);

/* Colour-ordered partial amplitudes A(sigma) of one event at helicity h,
 * out[ncolor][2] (re, im).  For ee->mumu (one colour flow) out[0] is the full
 * amplitude.  If gauge_leg >= 0, the polarisation vector of that (gluon) leg
 * is replaced by its momentum k/k^0: every partial amplitude must vanish. */
int oracle_partial_amps(int proc, const oracle_params* p, const double* mom, int hel,
                        int gauge_leg, double* out);

/* Colour-dressed amplitude of one event for explicit colours: colours[g] in
 * 0..7 for each gluon g (gluon numbering above), then the top colour i_t and
 * antitop colour j_tbar in 0..2.  out[2] = (re, im). */
int oracle_dressed_amp(int proc, const oracle_params* p, const double* mom, int hel,
                       const int* colours, double* out);

/* Colour factors c_sigma = (t^{a_sigma1} ... t^{a_sigman})_{i_t j_tbar} of the
 * colour-flow basis for explicit colours (same layout as above), out[n!][2]. */
int oracle_colour_basis(int ngluons, const int* colours, double* out);

/* Colour matrix C[sigma][tau] = sum_colours conj(c_sigma) c_tau, by brute
 * force over explicit Gell-Mann matrices, out[n!][n!]. */
int oracle_colour_matrix(int ngluons, double* out);

/* Phase-space points with counter-based random numbers (Philox4x32-10):
 * the four uniforms per final particle (cos theta, phi, two energy factors),
 * out[nevt][nfinal][4], and RAMBO momenta out[nevt][nfinal+2][4] (beams on
 * +-z at sqrt_s/2 each). */
int oracle_uniforms(int64_t nevt, int nfinal, uint64_t seed, double* out);
int oracle_rambo(int64_t nevt, int nfinal, const double* masses, double sqrt_s, uint64_t seed, double* out);

/* Importance-sampled phase-space points (sequential two-body splitting with
 * beam-peaked polar angles and soft-favouring remainder masses; the mapping
 * is spelled out in oracle.cpp) and their phase-space weights:
 * out[nevt][nfinal+2][4], weight[nevt]. */
int oracle_sample(int64_t nevt, int nfinal, const double* masses, double sqrt_s, uint64_t seed, double* out,
                  double* weight);

#ifdef __cplusplus
}
#endif
#endif
