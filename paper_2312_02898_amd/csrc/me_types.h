// Types shared by the runtime and the generated kernels (internal; the public
// interface is include/me.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {

enum { ME_MODE_FP64 = 0, ME_MODE_MIXED = 1, ME_MODE_MIXED_VALU = 2, ME_MODE_MIXED_MFMA32 = 3, ME_MODE_MIXED_MFMA16 = 4,
       ME_MODE_MIXED_MFMABF16 = 5 };

// Kernel argument block (passed by value; lives in the kernarg segment).
struct MeParams {
  double gs;        // strong coupling g_s = sqrt(4 pi alpha_s)
  double ea;        // photon-fermion coupling -e Q (Q = -1 for the leptons)
  double gzl, gzr;  // Z-lepton couplings -e cL, -e cR
  double mz, wz;    // Z mass and width
  double mt, wt;    // top mass and width (s-channel propagators)
  double wt_tchan;  // top width in t-channel propagators (0 in zero-width mode)
  // weighted-event epilogue (w_fac NULL: none): w_out[e] = max(|M|^2_e w_fac[e], 0)
  // when w_out is set, and their maximum as the bit pattern in *w_max
  const double* w_fac;
  double* w_out;
  unsigned long long* w_max;
  int32_t nhel;     // number of helicity configurations in hel[]
  int32_t pad;
  uint8_t hel[128]; // helicity configurations: bit i = leg i has helicity +1
};

// Launch of one process's kernels.  ws / ws_bytes: device workspace for the
// forms that need one (the split form); NULL lets the launch take it from the
// stream-ordered allocator.  0 on success, -1 bad arguments, -2 launch
// failure, -3 workspace allocation failed or too small.
typedef int (*LaunchFn)(int mode, const double* mom, int64_t nevt, double* out, double* out_hel,
                        const MeParams* prm, hipStream_t stream, void* ws, int64_t ws_bytes);
// Device workspace bytes a launch of nevt events with nhel helicities needs
// when it may use at most cap bytes (cap <= 0: the launch's own default);
// 0 for the forms that need none.
typedef int64_t (*WorkspaceFn)(int mode, int64_t nevt, int nhel, int64_t cap);

struct ProcessEntry {
  const char* name;
  const char* process;
  int npar, ncolor, nhel, ndiagrams, iden, colour_den;
  long flops_per_hel;  // algorithmic flops of one helicity of one event
  int massive_top;     // legs 2 and 3 carry the top mass
  int alphas_power;    // |M|^2 is proportional to alpha_s^alphas_power
  LaunchFn launch;
  WorkspaceFn workspace;
};

}  // namespace me
