// Serving runtime of the C ABI (me_server_* in include/me.h): the scheduling
// core of server_core.hpp driven by a HIP executor.  Each slot owns a HIP
// stream and a completion event; device memory for requests comes from one
// arena of budget_bytes, mirrored by a pinned host arena used for staging, so
// an admitted request costs no allocation: host copy into pinned staging,
// async H2D, me_compute, async D2H, event record, all on the slot's stream
// (a request above kServePieceFlops runs me_compute in pieces, the next one
// enqueued when the previous has completed).
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "handle.hpp"
#include "me.h"
#include "server_core.hpp"

namespace {

// A request above this estimated work runs in pieces of whole 2^14-event
// chunks (the split form's), one piece's kernels in its stream at a time
// (a piece of g g > t t~ g g g: about 17 ms mixed, 34 ms FP64); everything
// else runs whole.
constexpr int64_t kServePieceFlops = int64_t(200) * 1000 * 1000 * 1000;
constexpr int64_t kServePieceAlign = int64_t(1) << 14;

struct HipExec {
  int device = 0;
  char* d_arena = nullptr;
  char* h_arena = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<int> launch_ok;
  // a request in flight on a slot: its region and the next event to launch
  struct InFlight {
    me::Request req;
    int64_t off = 0, next = 0, piece = 0;
  };
  std::vector<InFlight> inflight;

  // Events per piece: the whole request, or whole chunks worth about
  // kServePieceFlops.  Pieces keep the hardware queue that a slot's stream
  // shares with other slots from holding a long request's whole kernel
  // sequence, behind which a small request would wait.
  static int64_t piece_events(const me::Request& r) {
    if (r.cost <= kServePieceFlops || r.nevt <= kServePieceAlign) return r.nevt;
    const int64_t per_event = r.cost / r.nevt > 0 ? r.cost / r.nevt : 1;
    int64_t n = (kServePieceFlops / per_event + kServePieceAlign - 1) / kServePieceAlign * kServePieceAlign;
    if (n < kServePieceAlign) n = kServePieceAlign;
    return n < r.nevt ? n : r.nevt;
  }
  // enqueues events [f.next, f.next + n) and, after the last piece, the copy
  // of the results; records the slot's event
  bool enqueue_piece(int slot) {
    InFlight& f = inflight[size_t(slot)];
    const me::Request& r = f.req;
    const int64_t n = r.nevt - f.next < f.piece ? r.nevt - f.next : f.piece;
    double* d_mom = reinterpret_cast<double*>(d_arena + f.off) + f.next * 4 * r.npar;
    double* d_out = reinterpret_cast<double*>(d_arena + f.off + out_offset(r)) + f.next;
    void* d_ws = r.ws_bytes > 0 ? d_arena + f.off + ws_offset(r) : nullptr;
    hipStream_t s = streams[size_t(slot)];
    bool ok = me::compute_on(static_cast<me_handle>(r.handle), d_mom, n, d_out, s, d_ws, r.ws_bytes) == ME_OK;
    f.next += n;
    if (ok && f.next == r.nevt)
      ok = hipMemcpyAsync(h_arena + f.off + out_offset(r), d_arena + f.off + out_offset(r), size_t(r.nevt) * 8,
                          hipMemcpyDeviceToHost, s) == hipSuccess;
    return ok && hipEventRecord(events[size_t(slot)], s) == hipSuccess;
  }

  static int64_t out_offset(const me::Request& r) { return r.nevt * int64_t(32) * r.npar; }
  // the request's region: momenta, results, then its process's workspace
  static int64_t ws_offset(const me::Request& r) { return me::Arena::round(me::ServerCore<HipExec>::io_bytes(r)); }

  bool launch(int slot, me::Request& r, int64_t off) {
    (void)hipSetDevice(device);
    launch_ok[slot] = 0;
    const size_t in_bytes = size_t(r.nevt) * 32 * r.npar;
    std::memcpy(h_arena + off, r.h_mom, in_bytes);
    hipStream_t s = streams[slot];
    InFlight& f = inflight[size_t(slot)];
    f.req = r;
    f.off = off;
    f.next = 0;
    f.piece = piece_events(r);
    bool ok = hipMemcpyAsync(d_arena + off, h_arena + off, in_bytes, hipMemcpyHostToDevice, s) == hipSuccess;
    ok = ok && enqueue_piece(slot);
    if (!ok) {
      // the core frees the region at once: nothing queued above may still
      // be reading or writing it
      (void)hipStreamSynchronize(s);
      return false;
    }
    launch_ok[slot] = 1;
    return true;
  }
  // the slot's work is done when its last piece and the copy of the results
  // have completed; a completed earlier piece starts the next one
  bool done(int slot) {
    if (hipEventQuery(events[slot]) == hipErrorNotReady) return false;
    InFlight& f = inflight[size_t(slot)];
    if (!launch_ok[slot] || f.next >= f.req.nevt) return true;
    if (!enqueue_piece(slot)) {
      (void)hipStreamSynchronize(streams[slot]);
      launch_ok[slot] = 0;   // finish() reports the failure
      return true;
    }
    return false;
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

// Requests above this estimated work (flop) are large: about 1 ms of the
// g g > t t~ g g g split form or of 14 000 g g > t t~ g g events.
constexpr int64_t kServeLargeFlops = int64_t(20) * 1000 * 1000 * 1000;

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
  ex.inflight.assign(size_t(n_slots), HipExec::InFlight{});
  if (!ok) {
    for (auto st : ex.streams) (void)hipStreamDestroy(st);
    for (auto ev : ex.events) (void)hipEventDestroy(ev);
    if (ex.d_arena) (void)hipFree(ex.d_arena);
    if (ex.h_arena) (void)hipHostFree(ex.h_arena);
    delete s;
    return ME_EHIP;
  }
  s->ws_cap = budget_bytes / 4 < kServeWorkspaceCap ? budget_bytes / 4 : kServeWorkspaceCap;
  s->core.reset(new me::ServerCore<HipExec>(ex, budget_bytes, n_slots, 16, kServeLargeFlops));
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
  // estimated device work: the process's algorithmic flops per helicity x
  // good helicities x events
  r.cost = nevt * int64_t(h->proc->flops_per_hel) * h->kp.nhel;
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
  st->passed_large = x.passed_large;
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
