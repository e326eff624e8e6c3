// replay.cpp -- serving client driver (libmg_clients.so): replays an arrival
// trace against an mg_server from many client threads at once, so that the
// server sees concurrent mg_server_submit calls at the trace's rate.
//
// Client thread c submits, in trace order, the requests whose client index is
// c, each at its scheduled arrival (sleeping until 200 us before it, then
// spinning on the server's clock), stamped with that arrival so that latency
// counts from the schedule (open loop: a late submission counts against the
// latency); a full queue is retried until it accepts.  After its last
// submission the thread waits for each of its tickets.
#include <algorithm>
#include <chrono>
#include <thread>
#include <vector>

#include "mg_clients.h"

extern "C" {

// n requests; client[i] in [0, n_clients), at_ns[i] = arrival offset from t0_ns
// (non-decreasing per client), reqs[i] the request (its arrival_ns is
// overwritten).  Writes status[i] (submit status if not MG_OK, else the wait
// status), latency_s[i] (arrival -> result in out, or -1) and lag_ns[i]
// (submission time - scheduled arrival).  Returns 0, or -1 for bad arguments.
int mgc_replay(mg_server* srv, int32_t n_clients, int64_t n, const int32_t* client,
               const uint64_t* at_ns, mg_request* reqs, uint64_t t0_ns, int32_t* status,
               double* latency_s, int64_t* lag_ns) {
  if (!srv || n_clients < 1 || n < 0 || (n > 0 && (!client || !at_ns || !reqs || !status ||
                                                   !latency_s || !lag_ns)))
    return -1;
  std::vector<std::vector<int64_t>> mine(n_clients);
  for (int64_t i = 0; i < n; ++i) {
    if (client[i] < 0 || client[i] >= n_clients) return -1;
    mine[client[i]].push_back(i);
  }
  auto run = [&](int c) {
    std::vector<uint64_t> tickets(mine[c].size(), 0);
    for (size_t k = 0; k < mine[c].size(); ++k) {
      const int64_t i = mine[c][k];
      const uint64_t at = t0_ns + at_ns[i];
      for (;;) {
        const uint64_t now = mg_clock_ns();
        if (now >= at) break;
        if (at - now > 300000)
          std::this_thread::sleep_for(std::chrono::nanoseconds(at - now - 200000));
      }
      reqs[i].arrival_ns = at;
      lag_ns[i] = (int64_t)(mg_clock_ns() - at);
      mg_status st;
      while ((st = mg_server_submit(srv, &reqs[i], &tickets[k])) == MG_ERR_BUSY)
        std::this_thread::yield();
      status[i] = st;
      latency_s[i] = -1.0;
      if (st != MG_OK) tickets[k] = 0;
    }
    for (size_t k = 0; k < mine[c].size(); ++k) {
      if (!tickets[k]) continue;
      const int64_t i = mine[c][k];
      double lat = -1.0;
      status[i] = mg_server_wait(srv, tickets[k], -1, &lat);
      latency_s[i] = lat;
    }
  };
  std::vector<std::thread> th;
  for (int c = 0; c < n_clients; ++c) th.emplace_back(run, c);
  for (auto& t : th) t.join();
  return 0;
}

}  // extern "C"
