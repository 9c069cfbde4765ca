"""The process compiler's output, compiled for the host CPU, against the oracle.

The generated straight-line programs (``csrc/gen/<process>_proc.inc``) and
the device functions they call (``csrc/helas.hpp``) are plain C++ apart from
HIP qualifiers and empty ``asm`` barriers.  Compiled with g++ behind a small
shim (qualifiers defined away, barriers dropped), they evaluate |M|^2 on the
CPU: the jamps of every helicity (FP64 and FP32 schedules) and the colour
sum with the integer colour matrix; a form whose kernel caches its
propagator factors and polarisation bases per event runs through a host
stand-in of that cache.  This pins the diagram enumeration, colour decomposition, schedule
(recomputation, evictions, jamp write-backs of the split form) and code
emission against the oracle without a GPU.  The GPU kernels themselves are
covered by the ``gpu`` tests.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2312_02898_amd.inputs import CONFIGS, config_events

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2312_02898_amd", "csrc")

SHIM = r"""
#pragma once
#include <cmath>
#include <cstdint>
#define __device__
#define __host__
#define __forceinline__ inline
#define __constant__
#define __global__
#define __launch_bounds__(x)
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
struct double2 { double x, y; };
typedef int hipStream_t;
using std::sqrt; using std::fabs; using std::fma; using std::copysign;
"""

MAIN = r"""
#include <cstdio>
#include <vector>
#include "helas.hpp"
#include "me_types.h"
namespace me {
template <class T> inline mom<T> neg(const mom<T>& k) { return mom<T>{{-k.k[0], -k.k[1], -k.k[2], -k.k[3]}}; }
template <class T> inline cx<T> prop_den(double k2, double m, double w) {
  const double a = k2 - m * m, b = m * w;
  const double r = 1.0 / (a * a + b * b);
  return cx<T>{T(a * r), T(-b * r)};
}
template <class T> inline void jw_store(cx<T>* jw, int64_t off, cx<T> v) { jw[off] = v; }
template <class T> inline void jw_add(cx<T>* jw, int64_t off, cx<T> v) { jw[off] = jw[off] + v; }
}
#include PROC_INC
using namespace me;
using P = PROC;
using T = EMU_T;
template <int J, class Q = P> void parts(const double (&p)[P::NPAR][4], unsigned h, const MeParams& prm, cx<T>* X) {
  constexpr int N = sizeof(T) == 8 ? Q::NPARTS_F64 : Q::NPARTS_F32;
  constexpr int NQ = sizeof(T) == 8 ? Q::QLDS_F64 : Q::QLDS_F32;
  // stands in for the part kernel's LDS jamp slots (this lane's row)
  static cx<T> qb[NQ > 0 ? NQ : 1];
  if constexpr (J < N) { Q::template part<T, J>(p, h, prm, X, 1, qb); parts<J + 1, Q>(p, h, prm, X); }
}
// stands in for the kernel's per-event LDS cache of propagator factors
// stands in for the FP64 kernel's per-event light-cone cache
struct HostLcCache {
  static constexpr bool kCached = false;
  static constexpr bool kMom = false;
  static constexpr bool kLc = true;
  double v[64];
  int npair0;
  double lcs(int k) const { return v[k]; }
  double pair(int k) const { return v[npair0 + k]; }
  void set_lcs(int k, double x) { v[k] = x; }
  void set_pair(int k, double x) { v[npair0 + k] = x; }
};
template <class T> struct HostKinCache {
  static constexpr bool kCached = true;
  static constexpr bool kMom = true;   // momentum sums and spinors too, where the form caches them
  static constexpr bool kLc = false;
  mom<T> km[64];
  wf<T> sps[16][2];
  mom<T> k(int s) const { return km[s]; }
  mom<T> k_opq(int s) const { return km[s]; }
  wf<T> sp(int j, int lam) const { return sps[j][lam > 0]; }
  wf<T> sp_opq(int j, int lam) const { return sp(j, lam); }
  void set_k(int s, const mom<T>& v) { km[s] = v; }
  void set_sp(int j, int lam, const wf<T>& w) { sps[j][lam > 0] = w; }
  double lcs(int) const { return 0.0; }
  double pair(int) const { return 0.0; }
  T re[64];
  cx<T> cxs[64];
  T r(int s) const { return re[s]; }
  cx<T> c(int s) const { return cxs[s]; }
  T r_opq(int s) const { return re[s]; }
  cx<T> c_opq(int s) const { return cxs[s]; }
  void set_r(int s, T v) { re[s] = v; }
  void set_c(int s, cx<T> v) { cxs[s] = v; }
  T eb[16][5];
  epsw<T> eps(int j, int lam, bool cj) const { return eps_from_base<T>(eb[j][0], eb[j][1], eb[j][2], eb[j][3], eb[j][4], lam, cj); }
  epsw<T> eps_opq(int j, int lam, bool cj) const { return eps(j, lam, cj); }
  void set_eps(int j, T a0, T a1, T a2, T b0, T b1) { eb[j][0] = a0; eb[j][1] = a1; eb[j][2] = a2; eb[j][3] = b0; eb[j][4] = b1; }
};
// a template, so that the branch for the other form is discarded
template <class Q>
void jamps(const double (&p)[Q::NPAR][4], unsigned h, const MeParams& prm, cx<T>* J) {
  if constexpr (Q::SPLIT) {
    for (int k = 0; k < Q::NCOLOR; ++k) J[k] = cx<T>{T(1e30), T(1e30)};   // every jamp must be stored
    parts<0>(p, h, prm, J);
  } else if constexpr (sizeof(T) == 8 && Q::KC_RE_F64 + Q::KC_CX_F64 + Q::KC_EPS_F64 > 0) {
    static_assert(Q::KC_RE_F64 <= 64 && Q::KC_CX_F64 <= 64 && Q::KC_EPS_F64 <= 16, "host cache too small");
    HostKinCache<T> dc;
    for (int s = 0; s < 64; ++s) { dc.re[s] = T(1e30); dc.cxs[s] = cx<T>{T(1e30), T(1e30)}; }
    for (int s = 0; s < 16; ++s) for (int c = 0; c < 5; ++c) dc.eb[s][c] = T(1e30);
    Q::template den_fill_f64<T>(p, prm, dc);
    Q::template amplitudes_f64<T>(p, h, prm, J, dc);
  } else if constexpr (sizeof(T) == 8 && Q::FP64_LDS_JAMPS) {
    // the FP64 kernel with LDS jamps reads its light-cone invariants from a cache
    HostLcCache lc;
    lc.npair0 = Q::LC_LEGS;
    for (int s = 0; s < 64; ++s) lc.v[s] = 1e30;
    Q::lc_fill(p, prm, lc);
    Q::template amplitudes_f64<T>(p, h, prm, J, lc);
  } else if constexpr (sizeof(T) == 8) {
    Q::template amplitudes_f64<T>(p, h, prm, J);
  } else if constexpr (Q::KC_RE_F32 + Q::KC_CX_F32 + Q::KC_EPS_F32 > 0) {
    static_assert(Q::KC_RE_F32 <= 64 && Q::KC_CX_F32 <= 64 && Q::KC_EPS_F32 <= 16, "host cache too small");
    static_assert(Q::KC_MOM_F32 <= 64 && Q::KC_SP_F32 <= 16, "host cache too small");
    HostKinCache<T> dc;
    for (int s = 0; s < 64; ++s) { dc.re[s] = T(1e30); dc.cxs[s] = cx<T>{T(1e30), T(1e30)}; }
    for (int s = 0; s < 64; ++s) for (int c = 0; c < 4; ++c) dc.km[s].k[c] = T(1e30);
    for (int s = 0; s < 16; ++s) for (int l = 0; l < 2; ++l) for (int c = 0; c < 4; ++c) dc.sps[s][l].c[c] = cx<T>{T(1e30), T(1e30)};
    for (int s = 0; s < 16; ++s) for (int c = 0; c < 5; ++c) dc.eb[s][c] = T(1e30);
    Q::template den_fill_f32<T>(p, prm, dc);
    Q::template amplitudes_f32<T>(p, h, prm, J, dc);
  } else {
    Q::template amplitudes_f32<T>(p, h, prm, J);
  }
}
int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  long n = 0;
  if (fread(&n, 8, 1, f) != 1) return 1;
  std::vector<double> mom(n * P::NPAR * 4);
  if (fread(mom.data(), 8, mom.size(), f) != mom.size()) return 1;
  fclose(f);
  MeParams prm{};
  prm.gs = std::sqrt(4 * M_PI * 0.118);
  prm.mt = 173.0; prm.wt = 1.49; prm.wt_tchan = 0.0;
  for (long e = 0; e < n; ++e) {
    double p[P::NPAR][4];
    // on the mass shell, as the kernels load them
    for (int i = 0; i < P::NPAR; ++i) {
      for (int c = 1; c < 4; ++c) p[i][c] = mom[(e * P::NPAR + i) * 4 + c];
      const double m2 = (P::MASSIVE >> i & 1u) ? prm.mt * prm.mt : 0.0;
      p[i][0] = std::copysign(std::sqrt(m2 + p[i][1] * p[i][1] + p[i][2] * p[i][2] + p[i][3] * p[i][3]),
                              mom[(e * P::NPAR + i) * 4]);
    }
    double acc = 0.0;
    for (unsigned h = 0; h < P::NHEL; ++h) {
      cx<T> J[P::NCOLOR];
      jamps<P>(p, h, prm, J);
      for (int k = 0; k < P::NCOLOR; ++k)
        for (int l = 0; l < P::NCOLOR; ++l)
          acc += P::cmat()[k * P::NCOLOR + l] * (double(J[k].r) * J[l].r + double(J[k].i) * J[l].i);
    }
    printf("%.17g\n", acc * P::coupling_factor(prm) / (P::CDEN * P::IDEN));
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def emu_dir(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("emu")
    (d / "hip").mkdir()
    (d / "hip" / "hip_runtime.h").write_text(SHIM)
    with open(os.path.join(CSRC, "helas.hpp")) as f:
        helas = [ln for ln in f if "asm volatile" not in ln]
    (d / "helas.hpp").write_text("".join(helas))
    shutil.copy(os.path.join(CSRC, "me_types.h"), d / "me_types.h")
    (d / "main.cpp").write_text(MAIN)
    return d


@pytest.mark.parametrize("form", ["f64", "f32"])
@pytest.mark.parametrize("proc,nevt", [("uutt", 64), ("uxutt", 64), ("uuttg", 48), ("ugttu", 48), ("guxttux", 48), ("ggttg", 64), ("ggttgg", 24), ("ggttggg", 3),
                                       ("uuttgg", 24), ("uxuttgg", 16), ("ugttug", 24), ("guttug", 16),
                                       ("uxgttuxg", 16), ("guxttuxg", 16), ("ggttuux", 24), ("uuttuux", 32),
                                       ("uuttddx", 32), ("uuttuu", 32), ("udttud", 32), ("uxuxttuxux", 32)])
def test_generated_program_matches_oracle(oracle_lib, emu_dir, proc, nevt, form):
    """FP64 schedule: within 1e-12 of the oracle; FP32 schedule (FP32
    vertices, FP64 kinematics): median <= 1e-5, max <= 1e-3."""
    inc = os.path.join(CSRC, "gen", f"{proc}_proc.inc")
    if not os.path.exists(inc):
        pytest.skip("generated sources missing (run the build)")
    exe = emu_dir / f"emu_{proc}_{form}"
    # the cmat() accessor reads a __constant__ array: a plain global on the host
    r = subprocess.run(["g++", "-O1", "-std=c++17", f"-I{emu_dir}", f'-DPROC_INC="{inc}"', f"-DPROC=Proc_{proc}",
                        "-DEMU_T=" + ("double" if form == "f64" else "float"),
                        str(emu_dir / "main.cpp"), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    mom = config_events(proc, nevt)
    fin = emu_dir / f"mom_{proc}.bin"
    with open(fin, "wb") as f:
        np.array([nevt], dtype=np.int64).tofile(f)
        mom.tofile(f)
    out = subprocess.run([str(exe), str(fin)], capture_output=True, text=True, check=True).stdout.split()
    got = np.array([float(x) for x in out])
    ref = oracle_lib.me(CONFIGS[proc][0], mom)
    rel = np.abs(got / ref - 1.0)
    print(f"  {proc} {form}: host-compiled program vs oracle max rel {rel.max():.3e} median {np.median(rel):.3e}")
    if form == "f64":
        assert rel.max() <= 1e-12
    else:
        assert np.median(rel) <= 1e-5 and rel.max() <= 1e-3
