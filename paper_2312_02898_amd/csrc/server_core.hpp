// Serving core: a persistent request loop with admission by device-memory
// footprint and a fixed number of execution slots (continuous batching of
// uneven |M|^2 requests from several processes).
//
// A request's footprint is everything its device work touches: momenta,
// results and the workspace its process needs (the split form's jamp
// workspace), all carved from one arena of the server's budget.  Requests
// are admitted in arrival order as soon as a slot is free and the arena can
// hold the head's footprint.  When the head does not fit (it waits for
// memory, not for a slot), later requests that fit may pass it, but at most
// max_bypass of them per head: after that the queue is strictly in order
// until the head is admitted, so the head's wait is bounded by the service
// of the work already admitted.  With a cost threshold, large requests (by
// estimated device work) may hold at most half of the slots, the rest being
// kept for small ones, and small requests pass a large head that waits for
// such a slot: a small request then never queues behind long ones.  Requests admitted while others are in
// flight run concurrently on their own slots.  The executor does the device
// work; the core only does bookkeeping, so it is independent of HIP and can
// be driven by a fake executor on the CPU.
//
//   struct Executor {
//     // start the request's work on `slot`; false on launch failure, and
//     // then nothing of the request may still be in flight on the slot
//     bool launch(int slot, Request& r, int64_t offset);
//     // non-blocking completion test of the work on `slot`
//     bool done(int slot);
//     // finish a completed request (copy results out); false on failure
//     bool finish(int slot, Request& r, int64_t offset);
//   };
#pragma once
#include <stdint.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

namespace me {

struct Request {
  int64_t ticket = 0;
  void* handle = nullptr;          // me_handle (opaque here)
  const double* h_mom = nullptr;   // host input  [nevt][npar][4]
  double* h_out = nullptr;         // host output [nevt]
  int64_t nevt = 0;
  int32_t npar = 0;
  int64_t ws_bytes = 0;            // device workspace of the request's process (set by the submitter)
  int64_t cost = 0;                // estimated device work (flop; set by the submitter)
  bool large = false;              // cost above the server's threshold (set at submission)
  int64_t bytes = 0;               // device footprint: momenta, results and workspace
  std::chrono::steady_clock::time_point t_submit;
  std::chrono::steady_clock::time_point t_admit;   // slot and memory granted, work launched
};

struct TicketState {
  int done = 0;
  int status = 0;
  double latency_s = 0;   // submit -> completion
  double queue_s = 0;     // submit -> admission (the rest of the latency is service)
};

// First-fit allocator over [0, capacity) with 256-byte granules.
class Arena {
 public:
  explicit Arena(int64_t cap) : cap_(cap) { free_[0] = cap; }
  static int64_t round(int64_t b) { return (b + 255) & ~int64_t(255); }
  int64_t alloc(int64_t bytes) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        int64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_ += bytes;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = round(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t used() const { return used_; }
  int64_t capacity() const { return cap_; }

 private:
  int64_t cap_;
  int64_t used_ = 0;
  std::map<int64_t, int64_t> free_;
};

struct ServerStats {
  int64_t submitted = 0, completed = 0, failed = 0, rejected = 0, events_completed = 0;
  int64_t bypassed = 0;   // admissions past a head that waited for memory
  int64_t passed_large = 0;   // admissions past a large head that waited for a large-request slot
  int64_t bytes_in_use = 0, peak_bytes_in_use = 0;
  int32_t active_slots = 0, queued = 0;
};

template <class Exec>
class ServerCore {
 public:
  // momenta [nevt][npar][4] and results [nevt] precede the workspace in a
  // request's region
  static int64_t io_bytes(const Request& r) { return r.nevt * (int64_t(32) * r.npar + 8); }

  // large_cost > 0 splits requests into small and large by their cost: at
  // most nslots - small_slots large requests are in flight at once (small_slots
  // < 0: half of the slots), so small requests always find a slot instead of
  // queueing behind long ones; large requests take slots from the low end,
  // small ones from the high end.
  ServerCore(Exec& ex, int64_t budget, int nslots, int max_bypass = 16, int64_t large_cost = 0,
             int small_slots = -1)
      : ex_(ex), arena_(budget), slots_(nslots), max_bypass_(max_bypass), large_cost_(large_cost), stop_(false) {
    if (small_slots < 0) small_slots = nslots / 2;
    if (small_slots > nslots - 1) small_slots = nslots - 1;
    large_cap_ = large_cost > 0 ? nslots - small_slots : nslots;
    loop_ = std::thread([this] { run(); });
  }
  ~ServerCore() { shutdown(); }

  // 0 on success; -1 invalid, -3 larger than the whole budget.
  int submit(Request r, int64_t* ticket) {
    if (r.nevt <= 0 || !r.h_mom || !r.h_out || r.npar <= 0 || r.ws_bytes < 0) return -1;
    r.bytes = Arena::round(Arena::round(io_bytes(r)) + r.ws_bytes);
    r.large = large_cost_ > 0 && r.cost > large_cost_;
    std::lock_guard<std::mutex> lk(mu_);
    if (r.bytes > arena_.capacity()) {
      ++st_.rejected;
      return -3;
    }
    r.ticket = ++next_ticket_;
    r.t_submit = std::chrono::steady_clock::now();
    tickets_[r.ticket] = TicketState{};
    queue_.push_back(r);
    ++st_.submitted;
    *ticket = r.ticket;
    cv_.notify_all();
    return 0;
  }

  bool poll(int64_t ticket, TicketState* out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = tickets_.find(ticket);
    if (it == tickets_.end()) return false;
    *out = it->second;
    return true;
  }

  // true when done within timeout_s
  bool wait(int64_t ticket, double timeout_s, TicketState* out, bool* known) {
    std::unique_lock<std::mutex> lk(mu_);
    auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    *known = tickets_.count(ticket) != 0;
    if (!*known) return false;
    bool ok = done_cv_.wait_until(lk, deadline, [&] { return tickets_[ticket].done != 0; });
    *out = tickets_[ticket];
    return ok;
  }

  ServerStats stats() {
    std::lock_guard<std::mutex> lk(mu_);
    ServerStats s = st_;
    s.bytes_in_use = arena_.used();
    s.queued = int32_t(queue_.size());
    int act = 0;
    for (auto& sl : slots_) act += sl.busy ? 1 : 0;
    s.active_slots = act;
    return s;
  }

  void shutdown() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stop_) return;
      stop_ = true;
      cv_.notify_all();
    }
    if (loop_.joinable()) loop_.join();
  }

 private:
  struct Slot {
    bool busy = false;
    Request req;
    int64_t off = -1;
  };

  void complete(Slot& s, int status) {
    auto now = std::chrono::steady_clock::now();
    TicketState& t = tickets_[s.req.ticket];
    t.done = 1;
    t.status = status;
    t.latency_s = std::chrono::duration<double>(now - s.req.t_submit).count();
    t.queue_s = std::chrono::duration<double>(s.req.t_admit - s.req.t_submit).count();
    if (s.req.large) --large_active_;
    if (status == 0) {
      ++st_.completed;
      st_.events_completed += s.req.nevt;
    } else {
      ++st_.failed;
    }
    arena_.release(s.off, s.req.bytes);
    s.busy = false;
    s.off = -1;
  }

  // One pass: retire finished work, admit the queue head while possible.
  // Returns true if anything changed.
  bool step(std::unique_lock<std::mutex>& lk) {
    bool progress = false;
    for (size_t i = 0; i < slots_.size(); ++i) {
      Slot& s = slots_[i];
      if (!s.busy || !ex_.done(int(i))) continue;
      Request r = s.req;
      int64_t off = s.off;
      lk.unlock();
      bool ok = ex_.finish(int(i), r, off);
      lk.lock();
      complete(s, ok ? 0 : -4);
      progress = true;
    }
    while (!queue_.empty()) {
      bool any_free = false;
      for (auto& sl : slots_) any_free |= !sl.busy;
      if (!any_free) break;
      // the head if it may start now; else the first later request that may
      // (past a head that waits for memory at most max_bypass times; past a
      // large head that waits for a large-request slot freely: that costs
      // the head nothing, small requests never take those slots)
      size_t pick = 0;
      int64_t off = -1;
      const bool head_class_ok = class_ok(queue_.front());
      if (head_class_ok) off = arena_.alloc(queue_.front().bytes);
      if (off < 0) {
        if (head_class_ok && head_bypassed_ >= max_bypass_) break;   // strictly in order until the head is admitted
        // past a large head that waits for a slot, only into the slots
        // reserved for small requests: the head's slots stay for it
        if (!head_class_ok && free_slot_in(large_cap_, int(slots_.size())) < 0) break;
        for (size_t q = 1; q < queue_.size() && q <= kBypassWindow; ++q) {
          if (!class_ok(queue_[q]) || (!head_class_ok && queue_[q].large)) continue;
          off = arena_.alloc(queue_[q].bytes);
          if (off >= 0) { pick = q; break; }
        }
        if (off < 0) break;
        if (head_class_ok) {
          ++head_bypassed_;
          ++st_.bypassed;
        } else {
          ++st_.passed_large;
        }
      } else {
        head_bypassed_ = 0;
      }
      const int free_slot = slot_for(queue_[pick]);
      Slot& s = slots_[free_slot];
      s.req = queue_[pick];
      s.req.t_admit = std::chrono::steady_clock::now();
      queue_.erase(queue_.begin() + std::ptrdiff_t(pick));
      s.busy = true;
      s.off = off;
      if (s.req.large) ++large_active_;
      st_.peak_bytes_in_use = std::max(st_.peak_bytes_in_use, arena_.used());
      Request r = s.req;
      lk.unlock();
      bool ok = ex_.launch(free_slot, r, off);
      lk.lock();
      if (!ok) complete(s, -4);
      progress = true;
    }
    if (progress) done_cv_.notify_all();
    return progress;
  }

  void run() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      bool progress = step(lk);
      bool busy = false;
      for (auto& s : slots_) busy |= s.busy;
      if (stop_ && !busy && queue_.empty()) break;
      if (stop_ && !busy && !queue_.empty()) {
        // cannot happen (every queued request fits the arena when idle), but never spin forever
        while (!queue_.empty()) {
          tickets_[queue_.front().ticket] = TicketState{1, -6, 0.0};
          ++st_.failed;
          queue_.pop_front();
        }
        done_cv_.notify_all();
        break;
      }
      if (progress) continue;
      if (busy) {
        // device work in flight: poll at a short interval
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      } else {
        cv_.wait_for(lk, std::chrono::milliseconds(50));
      }
    }
  }

  // a request may start now as far as its class goes (a free slot of the
  // right kind exists: checked by the caller and slot_for)
  bool class_ok(const Request& r) const {
    if (r.large) return large_active_ < large_cap_ && free_slot_in(0, large_cap_) >= 0;
    return true;
  }
  int free_slot_in(int lo, int hi) const {
    for (int i = lo; i < hi; ++i)
      if (!slots_[size_t(i)].busy) return i;
    return -1;
  }
  // large requests: the lowest free slot; small ones: the highest
  int slot_for(const Request& r) const {
    if (r.large) return free_slot_in(0, large_cap_);
    for (int i = int(slots_.size()) - 1; i >= 0; --i)
      if (!slots_[size_t(i)].busy) return i;
    return -1;
  }

  // later requests looked at when the head does not fit
  static constexpr size_t kBypassWindow = 1024;

  Exec& ex_;
  Arena arena_;
  std::vector<Slot> slots_;
  int max_bypass_;
  int64_t large_cost_;
  int large_cap_ = 0;       // large requests in flight at most
  int large_active_ = 0;
  int head_bypassed_ = 0;   // requests admitted past the current head
  std::deque<Request> queue_;
  std::map<int64_t, TicketState> tickets_;
  ServerStats st_;
  int64_t next_ticket_ = 0;
  bool stop_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::thread loop_;
};

}  // namespace me
