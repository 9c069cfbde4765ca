// Multi-subprocess requests: one batch whose events belong to different
// subprocesses (channels) of the same final state, e.g. the g g, u u~ and
// u~ u channels of p p -> t t~, with an optional per-event strong coupling.
//
// The batch is partitioned by channel on the device (stable: events keep
// their input order within a channel), each channel's events are gathered
// into a contiguous block and evaluated by that channel's kernels, and the
// results are scattered back, rescaled by (alpha_s(e) / alpha_s,ref)^p: every
// diagram of these processes carries the same power of g_s, so |M|^2 scales
// exactly with alpha_s^p (p = 2 for 2 -> t tbar, one more per extra gluon).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace me {
namespace chan {

constexpr int kMaxChannels = 32;

struct Scale {
  double aref[kMaxChannels];   // alpha_s the channel's kernels run with
  int32_t power[kMaxChannels]; // power of alpha_s in |M|^2
};

// One allocation holds: perm[nevt] (int64), gathered results[nevt],
// gathered momenta[nevt][npar][4], per-block counts and offsets, totals, a
// flag for channel indices out of range.
struct Workspace {
  int64_t* perm;
  double* out;
  double* mom;
  int32_t* counts;
  int64_t* offs;
  int64_t* totals;
  int32_t* bad;
};
size_t workspace_bytes(int64_t nevt, int nch, int npar);
Workspace carve(void* base, int64_t nevt, int nch, int npar);

// Stable partition by channel; copies the per-channel totals and the
// out-of-range flag to the host (this synchronises the stream).
hipError_t partition(const int32_t* d_channel, int64_t nevt, int nch, const Workspace& w, int64_t* h_totals,
                     int32_t* h_bad, hipStream_t s);
// dst[i] = mom[perm[i]] for i < n (4 npar doubles per event)
hipError_t gather(const double* mom, const int64_t* perm, int64_t n, int npar, double* dst, hipStream_t s);
// out[perm[j]] = res[j] * (alphas ? (alphas[e] / aref[c])^power[c] : 1), c = channel[e]
hipError_t scatter(const double* res, const int64_t* perm, const int32_t* channel, const double* alphas,
                   const Scale& sc, int64_t nevt, double* out, hipStream_t s);

}  // namespace chan
}  // namespace me
