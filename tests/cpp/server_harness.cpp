// CPU driver of the serving core with a fake executor: each request
// "runs" for a synthetic service time, results are written by the host, and
// failures can be injected at launch or at finish.  Prints one JSON object.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "server_core.hpp"

using clk = std::chrono::steady_clock;

struct FakeExec {
  double service_s = 0.01;
  std::vector<double> service_of;   // per ticket (index ticket - 1), overrides service_s
  int fail_launch_ticket = -1, fail_finish_ticket = -1;
  std::vector<clk::time_point> t0;
  std::vector<int64_t> slot_ticket;
  std::mutex mu;
  std::vector<int64_t> admit_order;
  std::vector<std::pair<double, double>> intervals;   // (start, end) per finished request
  clk::time_point origin = clk::now();
  std::atomic<int> concurrent{0}, max_concurrent{0};

  explicit FakeExec(int nslots) : t0(nslots), slot_ticket(nslots, -1) {}
  bool launch(int slot, me::Request& r, int64_t) {
    std::lock_guard<std::mutex> lk(mu);
    admit_order.push_back(r.ticket);
    if (r.ticket == fail_launch_ticket) return false;
    t0[slot] = clk::now();
    slot_ticket[slot] = r.ticket;
    int c = ++concurrent;
    if (c > max_concurrent) max_concurrent = c;
    return true;
  }
  bool done(int slot) {
    const int64_t t = slot_ticket[slot];
    const double sv = t >= 1 && size_t(t) <= service_of.size() ? service_of[t - 1] : service_s;
    return std::chrono::duration<double>(clk::now() - t0[slot]).count() >= sv;
  }
  bool finish(int slot, me::Request& r, int64_t) {
    std::lock_guard<std::mutex> lk(mu);
    --concurrent;
    intervals.push_back({std::chrono::duration<double>(t0[slot] - origin).count(),
                         std::chrono::duration<double>(clk::now() - origin).count()});
    for (int64_t i = 0; i < r.nevt; ++i) r.h_out[i] = r.h_mom[i * 4 * r.npar] * 2.0;
    return r.ticket != fail_finish_ticket;
  }
};

// Requests with a device workspace, and a head that waits for memory.
//   "workspace": 12 requests of 1000 events (136 000 B of momenta and
//   results) plus 300 000 B of workspace each, 1 MiB budget, 8 slots: the
//   footprint with the workspace limits concurrency to two.
//   "bypass": three 400 kB requests (80 ms), then one of 900 kB that must
//   wait for all of them, then 40 small ones (40 kB, 5 ms): small ones pass
//   the waiting head at most max_bypass = 16 times, then the queue is in
//   order until the big one is admitted.
int run_footprint(const std::string& sc) {
  const int nslots = 8;
  const int64_t budget = 1 << 20;
  FakeExec ex(nslots);
  std::vector<int64_t> nevts, wss;
  if (sc == "workspace") {
    for (int i = 0; i < 12; ++i) { nevts.push_back(1000); wss.push_back(300000); ex.service_of.push_back(0.02); }
  } else {
    for (int i = 0; i < 3; ++i) { nevts.push_back(2000); wss.push_back(128000); ex.service_of.push_back(0.08); }
    nevts.push_back(1000); wss.push_back(764000); ex.service_of.push_back(0.01);
    for (int i = 0; i < 40; ++i) { nevts.push_back(100); wss.push_back(26000); ex.service_of.push_back(0.005); }
  }
  const int nreq = int(nevts.size());
  std::vector<std::vector<double>> in(nreq), out(nreq);
  std::vector<int64_t> tickets;
  std::vector<double> queue(nreq);
  std::vector<int> status(nreq);
  me::ServerStats st;
  {
    me::ServerCore<FakeExec> core(ex, budget, nslots);
    for (int i = 0; i < nreq; ++i) {
      in[i].assign(nevts[i] * 16, 0.0);
      for (int64_t e = 0; e < nevts[i]; ++e) in[i][e * 16] = double(i * 100000 + e);
      out[i].assign(nevts[i], -1.0);
      me::Request r;
      r.h_mom = in[i].data(); r.h_out = out[i].data(); r.nevt = nevts[i]; r.npar = 4; r.ws_bytes = wss[i];
      int64_t t = -1;
      if (core.submit(r, &t) != 0) return 2;
      tickets.push_back(t);
      if (sc == "bypass" && i == 2) std::this_thread::sleep_for(std::chrono::milliseconds(5));
    }
    for (int i = 0; i < nreq; ++i) {
      me::TicketState ts; bool known;
      bool ok = core.wait(tickets[i], 30.0, &ts, &known);
      status[i] = ok ? ts.status : 999;
      queue[i] = ts.queue_s;
    }
    st = core.stats();
  }
  int correct = 1;
  for (int i = 0; i < nreq; ++i)
    for (size_t e = 0; e < out[i].size(); ++e)
      if (out[i][e] != 2.0 * in[i][e * 16]) correct = 0;
  printf("{\"scenario\": \"%s\", \"correct\": %d, \"completed\": %lld, \"failed\": %lld, \"bypassed\": %lld,"
         " \"peak_bytes\": %lld, \"bytes_in_use\": %lld, \"budget\": %lld, \"max_concurrent\": %d, \"status\": [",
         sc.c_str(), correct, (long long)st.completed, (long long)st.failed, (long long)st.bypassed,
         (long long)st.peak_bytes_in_use, (long long)st.bytes_in_use, (long long)budget, ex.max_concurrent.load());
  for (int i = 0; i < nreq; ++i) printf("%s%d", i ? ", " : "", status[i]);
  printf("], \"queue\": [");
  for (int i = 0; i < nreq; ++i) printf("%s%.6f", i ? ", " : "", queue[i]);
  printf("], \"admit_order\": [");
  for (size_t i = 0; i < ex.admit_order.size(); ++i) printf("%s%lld", i ? ", " : "", (long long)ex.admit_order[i]);
  printf("]}\n");
  return 0;
}

// Large and small requests by estimated cost ("classes"): 8 slots, cost
// threshold 1000; 10 large requests (cost 5000, 150 ms) submitted first,
// then 30 small ones (cost 10, 5 ms).  At most 4 large ones run at once
// (half of the slots kept for small ones), the small ones start without
// waiting for the large ones, and every request completes.
int run_classes() {
  const int nslots = 8;
  FakeExec ex(nslots);
  std::vector<int64_t> costs;
  for (int i = 0; i < 10; ++i) { costs.push_back(5000); ex.service_of.push_back(0.15); }
  for (int i = 0; i < 30; ++i) { costs.push_back(10); ex.service_of.push_back(0.005); }
  const int nreq = int(costs.size());
  std::vector<std::vector<double>> in(nreq), out(nreq);
  std::vector<int64_t> tickets;
  std::vector<double> queue(nreq);
  std::vector<int> status(nreq);
  std::vector<int> live_large(nreq, 0);
  me::ServerStats st;
  int max_large = 0;
  {
    me::ServerCore<FakeExec> core(ex, int64_t(1) << 24, nslots, 16, 1000);
    for (int i = 0; i < nreq; ++i) {
      in[i].assign(100 * 16, 0.0);
      for (int64_t e = 0; e < 100; ++e) in[i][e * 16] = double(i * 1000 + e);
      out[i].assign(100, -1.0);
      me::Request r;
      r.h_mom = in[i].data(); r.h_out = out[i].data(); r.nevt = 100; r.npar = 4; r.cost = costs[i];
      int64_t t = -1;
      if (core.submit(r, &t) != 0) return 2;
      tickets.push_back(t);
    }
    // sample how many large requests run at once
    for (int k = 0; k < 400; ++k) {
      int large = 0;
      {
        std::lock_guard<std::mutex> lk(ex.mu);
        for (int sl = 0; sl < nslots; ++sl) {
          const int64_t t = ex.slot_ticket[size_t(sl)];
          if (t >= 1 && t <= 10 && ex.concurrent > 0) {
            const double age = std::chrono::duration<double>(clk::now() - ex.t0[size_t(sl)]).count();
            if (age < ex.service_of[size_t(t - 1)]) ++large;
          }
        }
      }
      if (large > max_large) max_large = large;
      std::this_thread::sleep_for(std::chrono::milliseconds(1));
    }
    for (int i = 0; i < nreq; ++i) {
      me::TicketState ts; bool known;
      bool ok = core.wait(tickets[i], 30.0, &ts, &known);
      status[i] = ok ? ts.status : 999;
      queue[i] = ts.queue_s;
    }
    st = core.stats();
  }
  int correct = 1;
  for (int i = 0; i < nreq; ++i)
    for (size_t e = 0; e < out[i].size(); ++e)
      if (out[i][e] != 2.0 * in[i][e * 16]) correct = 0;
  printf("{\"scenario\": \"classes\", \"correct\": %d, \"completed\": %lld, \"failed\": %lld, "
         "\"passed_large\": %lld, \"max_large\": %d, \"max_concurrent\": %d, \"status\": [",
         correct, (long long)st.completed, (long long)st.failed, (long long)st.passed_large, max_large,
         ex.max_concurrent.load());
  for (int i = 0; i < nreq; ++i) printf("%s%d", i ? ", " : "", status[i]);
  printf("], \"queue\": [");
  for (int i = 0; i < nreq; ++i) printf("%s%.6f", i ? ", " : "", queue[i]);
  printf("]}\n");
  return 0;
}

int main(int argc, char** argv) {
  std::string sc = argc > 1 ? argv[1] : "basic";
  if (sc == "workspace" || sc == "bypass") return run_footprint(sc);
  if (sc == "classes") return run_classes();
  int nslots = sc == "memory" ? 8 : 4;
  int64_t budget = sc == "memory" ? 300000 : (1 << 20);   // "memory": about 2 requests fit
  int nreq = sc == "overlap" ? 8 : 12;
  int64_t nevt = 1000;   // 1000 * (32*4 + 8) = 136000 B, ~7 fit in 1 MiB
  FakeExec ex(nslots);
  if (sc == "fail") { ex.fail_launch_ticket = 3; ex.fail_finish_ticket = 7; }
  if (sc == "overlap") ex.service_s = 0.05;
  std::vector<std::vector<double>> in(nreq), out(nreq);
  int64_t rejected_rc = 0;
  std::vector<int64_t> tickets;
  {
    me::ServerCore<FakeExec> core(ex, budget, nslots);
    auto tstart = clk::now();
    for (int i = 0; i < nreq; ++i) {
      int64_t n = nevt + 37 * i;
      in[i].assign(n * 16, 0.0);
      for (int64_t e = 0; e < n; ++e) in[i][e * 16] = double(i * 100000 + e);
      out[i].assign(n, -1.0);
      me::Request r;
      r.h_mom = in[i].data(); r.h_out = out[i].data(); r.nevt = n; r.npar = 4;
      int64_t t = -1;
      int rc = core.submit(r, &t);
      tickets.push_back(rc == 0 ? t : -1);
    }
    // oversize request and invalid request
    std::vector<double> big(16 * 100000), bigo(100000);
    me::Request rb; rb.h_mom = big.data(); rb.h_out = bigo.data(); rb.nevt = 100000; rb.npar = 4;
    int64_t tb;
    rejected_rc = core.submit(rb, &tb);
    me::Request bad; bad.h_mom = big.data(); bad.h_out = bigo.data(); bad.nevt = 0; bad.npar = 4;
    int bad_rc = core.submit(bad, &tb);
    std::vector<int> status(nreq);
    std::vector<double> lat(nreq);
    for (int i = 0; i < nreq; ++i) {
      me::TicketState st; bool known;
      bool ok = core.wait(tickets[i], 30.0, &st, &known);
      status[i] = ok ? st.status : 999;
      lat[i] = st.latency_s;
    }
    double wall = std::chrono::duration<double>(clk::now() - tstart).count();
    me::ServerStats s = core.stats();
    int correct = 1;
    for (int i = 0; i < nreq; ++i)
      if (status[i] == 0)
        for (size_t e = 0; e < out[i].size(); ++e)
          if (out[i][e] != 2.0 * in[i][e * 16]) correct = 0;
    printf("{\"scenario\": \"%s\", \"wall\": %.6f, \"rejected_rc\": %lld, \"bad_rc\": %d, \"correct\": %d,"
           " \"submitted\": %lld, \"completed\": %lld, \"failed\": %lld, \"rejected\": %lld,"
           " \"bytes_in_use\": %lld, \"peak_bytes\": %lld, \"budget\": %lld, \"max_concurrent\": %d,"
           " \"status\": [", sc.c_str(), wall, (long long)rejected_rc, bad_rc, correct,
           (long long)s.submitted, (long long)s.completed, (long long)s.failed, (long long)s.rejected,
           (long long)s.bytes_in_use, (long long)s.peak_bytes_in_use, (long long)budget, ex.max_concurrent.load());
    for (int i = 0; i < nreq; ++i) printf("%s%d", i ? ", " : "", status[i]);
    printf("], \"latency\": [");
    for (int i = 0; i < nreq; ++i) printf("%s%.6f", i ? ", " : "", lat[i]);
    printf("], \"admit_order\": [");
    for (size_t i = 0; i < ex.admit_order.size(); ++i) printf("%s%lld", i ? ", " : "", (long long)ex.admit_order[i]);
    printf("], \"tickets\": [");
    for (int i = 0; i < nreq; ++i) printf("%s%lld", i ? ", " : "", (long long)tickets[i]);
    printf("]}\n");
  }
  return 0;
}
