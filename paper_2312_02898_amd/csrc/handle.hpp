// The handle behind the C ABI (internal to the library).
#pragma once
#include <string>

#include "me.h"
#include "me_types.h"

struct me_handle_s {
  const me::ProcessEntry* proc;
  me_sm_params params;
  me::MeParams kp;        // kernel parameters incl. the good-helicity list
  int filtered;
  int device;
  int debug;              // ME_DEBUG set at creation: me_compute validates its momenta
};

namespace me {

// kernel mode of a handle's precision
inline int mode_of(const me_sm_params& p) {
  return p.precision == ME_MIXED          ? ME_MODE_MIXED
         : p.precision == ME_MIXED_VALU   ? ME_MODE_MIXED_VALU
         : p.precision == ME_MIXED_MFMA32 ? ME_MODE_MIXED_MFMA32
         : p.precision == ME_MIXED_MFMA16 ? ME_MODE_MIXED_MFMA16
         : p.precision == ME_MIXED_MFMABF16 ? ME_MODE_MIXED_MFMABF16
                                          : ME_MODE_FP64;
}

// Checks every event of a batch: finite components, E >= 0 and four-momentum
// balance (sum of incoming = sum of outgoing legs, legs 0 and 1 incoming)
// within 1e-9 of the incoming energy.  Returns the number of bad events
// (synchronises the stream); negative on a HIP error.
int64_t validate_momenta(const double* d_mom, int64_t nevt, int npar, hipStream_t s);

// me_compute with an optional device workspace for the processes that need
// one (ws == NULL: the stream-ordered allocator; otherwise ws_bytes of it,
// at least the handle's workspace(mode, nevt, nhel, ws_bytes)).  kp: the
// kernel parameters to launch with (NULL: the handle's own), e.g. the
// handle's with the weighted-event epilogue set.
me_status compute_on(me_handle h, const double* d_momenta, int64_t nevt, double* d_me, hipStream_t s, void* ws,
                     int64_t ws_bytes, const MeParams* kp = nullptr);

// Records code and message for me_last_error(); returns code.
me_status set_error(me_status code, const std::string& msg);

// me_compute_channels with an optional caller workspace: ws == NULL takes the
// workspace from the stream-ordered allocator; otherwise ws_bytes must cover
// chan::workspace_bytes() and every channel's launch must need no workspace
// of its own (nothing is allocated).  `who` prefixes error messages.
me_status compute_channels_on(const me_handle* handles, int32_t nchannels, const double* d_momenta,
                              const int32_t* d_channel, const double* d_alphas, int64_t nevt, double* d_me,
                              hipStream_t s, void* ws, int64_t ws_bytes, const char* who);

}  // namespace me
