"""The structurally-zero operand types of the vertex library, on the host.

An external massless vector is carried as epsw<T> (no time component, real z
component) and the vertex functions read vector operands through comp<M>(),
which yields the exact-zero type zero_t or the real-valued re<T> for those
components; a massless fermion line takes a zero_t mass and a re<T>
propagator factor.  Every vertex function called with these operands must
give the value it gives with the same operands written out as full complex
wavefunctions (time component 0, imaginary z component 0; mass 0;
propagator factor with imaginary part 0).  The device header is compiled
for the host with g++ behind the same shim as the generated programs.
"""
import os
import shutil
import subprocess

import pytest

from tests.test_codegen_host import SHIM

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2312_02898_amd", "csrc")

MAIN = r"""
#include <cstdio>
#include <cmath>
#include <random>
#include "helas.hpp"
using namespace me;
using T = double;
static std::mt19937_64 rng(12345);
static double u() { return std::uniform_real_distribution<double>(-1.0, 1.0)(rng); }
static cx<T> rc() { return cx<T>{u(), u()}; }
static wf<T> rw() { wf<T> w; for (int m = 0; m < 4; ++m) w.c[m] = rc(); return w; }
static mom<T> rk() { return mom<T>{{u(), u(), u(), u()}}; }
static epsw<T> re_eps() { epsw<T> e; e.c1 = rc(); e.c2 = rc(); e.c3 = u(); return e; }
static wf<T> full(const epsw<T>& e) {
  wf<T> w; w.c[0] = cx<T>{0.0, 0.0}; w.c[1] = e.c1; w.c[2] = e.c2; w.c[3] = cx<T>{e.c3, 0.0}; return w;
}
static double worst = 0.0;
static int checks = 0;
static void cmp(cx<T> a, cx<T> b, double scale) {
  const double d = std::fabs(a.r - b.r) + std::fabs(a.i - b.i);
  worst = std::fmax(worst, d / scale);
  ++checks;
}
static void cmpw(const wf<T>& a, const wf<T>& b, double scale) { for (int m = 0; m < 4; ++m) cmp(a.c[m], b.c[m], scale); }
static double nrm(const wf<T>& a) { double s = 0; for (int m = 0; m < 4; ++m) s += std::fabs(a.c[m].r) + std::fabs(a.c[m].i); return s; }
int main() {
  for (int t = 0; t < 200; ++t) {
    const epsw<T> E = re_eps(), F = re_eps(), G = re_eps();
    const wf<T> Ew = full(E), Fw = full(F), Gw = full(G);
    const wf<T> A = rw(), B = rw(), r = rw(), s = rw();
    const mom<T> K1 = rk(), K2 = rk(), K3 = rk();
    const cx<T> den = rc();
    const T m = 0.7, g = 0.9;
    // products
    cmp(dot(E, A), dot(Ew, A), 1.0); cmp(dot(A, E), dot(A, Ew), 1.0); cmp(dot(E, F), dot(Ew, Fw), 1.0);
    cmp(dot(K1, E), dot(K1, Ew), 1.0);
    // fermion-vector vertices with the vector external
    cmp(ffv_amp<T>(r, E, s, g, g), ffv_amp<T>(r, Ew, s, g, g), 1.0);
    cmpw(ffv_half_row<T>(r, E, g, g), ffv_half_row<T>(r, Ew, g, g), 1.0);
    cmpw(ffv_half_col<T>(E, s, g, g), ffv_half_col<T>(Ew, s, g, g), 1.0);
    cmpw(ffv_fin<T>(s, E, K1, m, den, g, g), ffv_fin<T>(s, Ew, K1, m, den, g, g), 1.0);
    cmpw(ffv_fout<T>(r, E, K1, m, den, g, g), ffv_fout<T>(r, Ew, K1, m, den, g, g), 1.0);
    // massless fermion line: zero_t mass and a real propagator factor
    const re<T> d0{den.r};
    const cx<T> d0c{den.r, 0.0};
    cmpw(ffv_fin<T>(s, A, K1, zero_t{}, d0, g, g), ffv_fin<T>(s, A, K1, T(0), d0c, g, g), 1.0);
    cmpw(ffv_fout<T>(r, E, K1, zero_t{}, d0, g, g), ffv_fout<T>(r, Ew, K1, T(0), d0c, g, g), 1.0);
    // three-gluon vertex: either or both operands external
    cmpw(vvv_v<T>(E, K1, A, K2, g), vvv_v<T>(Ew, K1, A, K2, g), 1.0);
    cmpw(vvv_v<T>(A, K1, E, K2, g), vvv_v<T>(A, K1, Ew, K2, g), 1.0);
    cmpw(vvv_v<T>(E, K1, F, K2, g), vvv_v<T>(Ew, K1, Fw, K2, g), 1.0);
    cmp(vvv_amp<T>(E, K1, A, K2, B, K3, g), vvv_amp<T>(Ew, K1, A, K2, B, K3, g), 1.0);
    cmp(vvv_amp<T>(A, K1, E, K2, F, K3, g), vvv_amp<T>(A, K1, Ew, K2, Fw, K3, g), 1.0);
    cmp(vvv_amp<T>(E, K1, F, K2, G, K3, g), vvv_amp<T>(Ew, K1, Fw, K2, Gw, K3, g), 1.0);
    // four-gluon pieces
    cmpw(vvvv_piece<T>(E, A, B), vvvv_piece<T>(Ew, A, B), 1.0);
    cmpw(vvvv_piece<T>(A, E, B), vvvv_piece<T>(A, Ew, B), 1.0);
    cmpw(vvvv_piece<T>(A, B, E), vvvv_piece<T>(A, B, Ew), 1.0);
    cmpw(vvvv_piece<T>(E, F, G), vvvv_piece<T>(Ew, Fw, Gw), 1.0);
    cmp(dot(E, vvvv_piece<T>(A, F, B)), dot(Ew, vvvv_piece<T>(A, Fw, B)), 1.0);
    // the polarisation vector from its cached base equals ext_eps
    double k[4] = {0, u(), u(), u()};
    k[0] = std::sqrt(k[1] * k[1] + k[2] * k[2] + k[3] * k[3]);
    for (int lam = -1; lam <= 1; lam += 2)
      for (int cj = 0; cj < 2; ++cj) {
        const EpsBase b = eps_base(k);
        const epsw<T> x = ext_eps<T>(k, lam, cj), y = eps_from_base<T>(b.a0, b.a1, b.a2, b.b0, b.b1, lam, cj);
        cmpw(full(x), full(y), 1.0);
        // and is transverse, normalised: k.eps = 0, eps.eps* = -1
        const wf<T> xw = full(x);
        wf<T> xc; for (int q = 0; q < 4; ++q) xc.c[q] = cconj(xw.c[q]);
        const mom<T> kk{{k[0], k[1], k[2], k[3]}};
        cmp(dot(kk, xw), cx<T>{0.0, 0.0}, 1.0);
        cmp(dot(xw, xc), cx<T>{-1.0, 0.0}, 1.0);
      }
  }
  std::printf("%d %.3e\n", checks, worst);
  return 0;
}
"""


def test_zero_types_match_full_operands(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    (tmp_path / "hip").mkdir()
    (tmp_path / "hip" / "hip_runtime.h").write_text(SHIM)
    with open(os.path.join(CSRC, "helas.hpp")) as f:
        (tmp_path / "helas.hpp").write_text("".join(ln for ln in f if "asm volatile" not in ln))
    (tmp_path / "main.cpp").write_text(MAIN)
    exe = tmp_path / "zt"
    r = subprocess.run(["g++", "-O1", "-std=c++17", f"-I{tmp_path}", str(tmp_path / "main.cpp"), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    checks, worst = int(out[0]), float(out[1])
    print(f"  {checks} comparisons, worst difference {worst:.3e}")
    assert checks > 4000
    # the same operations on the same values: equal up to rounding of the
    # few terms whose association the folding changes
    assert worst <= 1e-14
