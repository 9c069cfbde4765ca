// Serving runtime of the C ABI (me_server_* in include/me.h): the scheduling
// core of server_core.hpp driven by a HIP executor.  Each slot owns a HIP
// stream and a completion event; device memory for requests comes from one
// arena of budget_bytes, mirrored by a pinned host arena used for staging, so
// an admitted request costs no allocation: host copy into pinned staging,
// async H2D, me_compute, async D2H, event record, all on the slot's stream.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "handle.hpp"
#include "me.h"
#include "server_core.hpp"

namespace {

struct HipExec {
  int device = 0;
  char* d_arena = nullptr;
  char* h_arena = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<int> launch_ok;

  static int64_t out_offset(const me::Request& r) { return r.nevt * int64_t(32) * r.npar; }
  // the request's region: momenta, results, then its process's workspace
  static int64_t ws_offset(const me::Request& r) { return me::Arena::round(me::ServerCore<HipExec>::io_bytes(r)); }

  bool launch(int slot, me::Request& r, int64_t off) {
    (void)hipSetDevice(device);
    launch_ok[slot] = 0;
    const size_t in_bytes = size_t(r.nevt) * 32 * r.npar;
    std::memcpy(h_arena + off, r.h_mom, in_bytes);
    double* d_mom = reinterpret_cast<double*>(d_arena + off);
    double* d_out = reinterpret_cast<double*>(d_arena + off + out_offset(r));
    void* d_ws = r.ws_bytes > 0 ? d_arena + off + ws_offset(r) : nullptr;
    hipStream_t s = streams[slot];
    bool ok = hipMemcpyAsync(d_mom, h_arena + off, in_bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && me::compute_on(static_cast<me_handle>(r.handle), d_mom, r.nevt, d_out, s, d_ws, r.ws_bytes) == ME_OK;
    ok = ok && hipMemcpyAsync(h_arena + off + out_offset(r), d_out, size_t(r.nevt) * 8, hipMemcpyDeviceToHost,
                              s) == hipSuccess;
    ok = ok && hipEventRecord(events[slot], s) == hipSuccess;
    if (!ok) {
      // the core frees the region at once: nothing queued above may still
      // be reading or writing it
      (void)hipStreamSynchronize(s);
      return false;
    }
    launch_ok[slot] = 1;
    return true;
  }
  bool done(int slot) {
    hipError_t e = hipEventQuery(events[slot]);
    return e != hipErrorNotReady;
  }
  bool finish(int slot, me::Request& r, int64_t off) {
    if (!launch_ok[slot]) return false;
    if (hipEventSynchronize(events[slot]) != hipSuccess) return false;
    std::memcpy(r.h_out, h_arena + off + out_offset(r), size_t(r.nevt) * 8);
    return true;
  }
};

}  // namespace

// Workspace cap per request: a quarter of the budget, at most 128 MiB (the
// split form then runs its helicities in several passes over a smaller
// workspace; a request needs at least one helicity slot of it).
constexpr int64_t kServeWorkspaceCap = int64_t(128) << 20;

struct me_server_s {
  HipExec exec;
  int64_t ws_cap = 0;
  std::unique_ptr<me::ServerCore<HipExec>> core;
};

extern "C" {

me_status me_server_create(int64_t budget_bytes, int32_t n_slots, me_server* out) {
  if (!out || budget_bytes < 4096 || n_slots < 1 || n_slots > 64) return ME_EINVAL;
  me_server s = new (std::nothrow) me_server_s();
  if (!s) return ME_ENOMEM;
  HipExec& ex = s->exec;
  bool ok = hipGetDevice(&ex.device) == hipSuccess;
  ok = ok && hipMalloc(&ex.d_arena, size_t(budget_bytes)) == hipSuccess;
  ok = ok && hipHostMalloc(&ex.h_arena, size_t(budget_bytes), hipHostMallocDefault) == hipSuccess;
  for (int i = 0; ok && i < n_slots; ++i) {
    hipStream_t st;
    hipEvent_t ev;
    ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    if (ok) ex.streams.push_back(st);
    ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
    if (ok) ex.events.push_back(ev);
  }
  ex.launch_ok.assign(n_slots, 0);
  if (!ok) {
    for (auto st : ex.streams) (void)hipStreamDestroy(st);
    for (auto ev : ex.events) (void)hipEventDestroy(ev);
    if (ex.d_arena) (void)hipFree(ex.d_arena);
    if (ex.h_arena) (void)hipHostFree(ex.h_arena);
    delete s;
    return ME_EHIP;
  }
  s->ws_cap = budget_bytes / 4 < kServeWorkspaceCap ? budget_bytes / 4 : kServeWorkspaceCap;
  s->core.reset(new me::ServerCore<HipExec>(ex, budget_bytes, n_slots));
  *out = s;
  return ME_OK;
}

me_status me_server_submit(me_server s, me_handle h, const double* h_momenta, int64_t nevt, double* h_out,
                           int64_t* ticket) {
  if (!s || !h || !ticket) return ME_EINVAL;
  me_info_t info;
  if (me_info(h, &info) != ME_OK) return ME_EINVAL;
  me::Request r;
  r.handle = h;
  r.h_mom = h_momenta;
  r.h_out = h_out;
  r.nevt = nevt;
  r.npar = info.npar;
  // the device workspace of the request's process counts in its footprint
  r.ws_bytes = nevt > 0 ? h->proc->workspace(me::mode_of(h->params), nevt, h->kp.nhel, s->ws_cap) : 0;
  int rc = s->core->submit(r, ticket);
  if (rc == -1) return ME_EINVAL;
  if (rc == -3) return ME_ENOMEM;
  return ME_OK;
}

me_status me_server_poll(me_server s, int64_t ticket, int32_t* done, me_status* result, double* latency_s) {
  if (!s || !done) return ME_EINVAL;
  me::TicketState t;
  if (!s->core->poll(ticket, &t)) return ME_EINVAL;
  *done = t.done;
  if (result) *result = t.status;
  if (latency_s) *latency_s = t.latency_s;
  return ME_OK;
}

me_status me_server_wait(me_server s, int64_t ticket, double timeout_s, me_status* result, double* latency_s) {
  if (!s) return ME_EINVAL;
  me::TicketState t;
  bool known = false;
  bool ok = s->core->wait(ticket, timeout_s, &t, &known);
  if (!known) return ME_EINVAL;
  if (!ok) return ME_EBUSY;
  if (result) *result = t.status;
  if (latency_s) *latency_s = t.latency_s;
  return ME_OK;
}

me_status me_server_times(me_server s, int64_t ticket, double* queue_s, double* service_s) {
  if (!s || !queue_s || !service_s) return ME_EINVAL;
  me::TicketState t;
  if (!s->core->poll(ticket, &t)) return ME_EINVAL;
  if (!t.done) return ME_EBUSY;
  *queue_s = t.queue_s;
  *service_s = t.latency_s - t.queue_s;
  return ME_OK;
}

me_status me_server_stats(me_server s, me_server_stats_t* st) {
  if (!s || !st) return ME_EINVAL;
  me::ServerStats x = s->core->stats();
  st->submitted = x.submitted;
  st->completed = x.completed;
  st->failed = x.failed;
  st->rejected = x.rejected;
  st->events_completed = x.events_completed;
  st->bytes_in_use = x.bytes_in_use;
  st->peak_bytes_in_use = x.peak_bytes_in_use;
  st->active_slots = x.active_slots;
  st->queued = x.queued;
  st->bypassed = x.bypassed;
  return ME_OK;
}

me_status me_server_destroy(me_server s) {
  if (!s) return ME_EINVAL;
  s->core->shutdown();
  s->core.reset();
  HipExec& ex = s->exec;
  for (auto st : ex.streams) (void)hipStreamSynchronize(st);
  for (auto st : ex.streams) (void)hipStreamDestroy(st);
  for (auto ev : ex.events) (void)hipEventDestroy(ev);
  (void)hipFree(ex.d_arena);
  (void)hipHostFree(ex.h_arena);
  delete s;
  return ME_OK;
}

}  // extern "C"
