// serve_book.h -- host-only bookkeeping of the serving loop, shared by the
// client threads, the scheduler thread and the delivery threads:
//
//   TicketBook       a ticket per submitted request and its completion record
//                    (status, arrival and completion times); clients wait on it
//   AdmissionQueue   the bounded FIFO of requests not yet admitted, with the
//                    server's stop and failure state
//   DeliveryQueue    pieces of finished requests' results that delivery threads
//                    copy to the clients; a request completes with its last
//                    piece, a tick's result buffer is recycled with its last
//
// No HIP calls here, so the logic runs on the CPU under ThreadSanitizer.
#pragma once

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "mg.h"

namespace mg {

class TicketBook {
 public:
  // A new ticket for a request that arrived at `arrival_ns`.
  uint64_t open(uint64_t arrival_ns) {
    std::lock_guard<std::mutex> lk(mu_);
    const uint64_t t = next_++;
    rec_[t].arrival = arrival_ns;
    return t;
  }
  // Completes an open ticket with status st at done_ns and wakes its waiters;
  // an unknown or already completed ticket is left alone.
  void close(uint64_t ticket, mg_status st, uint64_t done_ns) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = rec_.find(ticket);
      if (it == rec_.end() || it->second.finished) return;
      it->second.done = done_ns;
      it->second.status = st;
      it->second.finished = true;
    }
    cv_.notify_all();
  }
  // Waits up to timeout_us (< 0: forever) for the ticket to complete.  The
  // first waiter to see it completed consumes it and gets its status (and the
  // arrival-to-completion time in *latency_s); MG_ERR_BUSY on timeout;
  // MG_ERR_INVALID for a ticket never issued or already consumed, also when
  // another waiter consumed it while this one waited.
  mg_status wait(uint64_t ticket, int64_t timeout_us, double* latency_s) {
    std::unique_lock<std::mutex> lk(mu_);
    if (rec_.find(ticket) == rec_.end()) return MG_ERR_INVALID;
    auto ready = [&] {
      auto it = rec_.find(ticket);
      return it == rec_.end() || it->second.finished;
    };
    if (timeout_us < 0)
      cv_.wait(lk, ready);
    else if (!cv_.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
      return MG_ERR_BUSY;
    auto it = rec_.find(ticket);
    if (it == rec_.end()) return MG_ERR_INVALID;
    const Record r = it->second;
    rec_.erase(it);
    if (latency_s) *latency_s = (double)(r.done - r.arrival) * 1e-9;
    return r.status;
  }
  // Whether the ticket was issued and has not completed yet.
  bool open_ticket(uint64_t ticket) const {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = rec_.find(ticket);
    return it != rec_.end() && !it->second.finished;
  }
  // Tickets issued and not yet consumed.
  size_t size() const {
    std::lock_guard<std::mutex> lk(mu_);
    return rec_.size();
  }

 private:
  struct Record {
    uint64_t arrival = 0, done = 0;
    mg_status status = MG_OK;
    bool finished = false;
  };
  mutable std::mutex mu_;
  std::condition_variable cv_;
  std::unordered_map<uint64_t, Record> rec_;
  uint64_t next_ = 1;
};

// Bounded FIFO of requests (owned pointers) waiting for admission.
template <class T>
class AdmissionQueue {
 public:
  enum class Admit { Take, Hold, Drop };

  explicit AdmissionQueue(size_t max_len) : max_(max_len) {}

  // Appends r unless the server failed (MG_ERR_DEVICE), is stopping or the
  // queue is full (MG_ERR_BUSY); `accept(r)` runs under the lock just before
  // the append (it issues the ticket), so tickets follow queue order.
  template <class Accept>
  mg_status push(T* r, Accept&& accept) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (failed_) return MG_ERR_DEVICE;
      if (stop_ || q_.size() >= max_) return MG_ERR_BUSY;
      accept(r);
      q_.push_back(r);
    }
    cv_.notify_one();
    return MG_OK;
  }
  // Blocks until a request is queued or the server stops or fails; false if
  // there is nothing to admit and never will be (stopped and empty, or failed).
  bool wait_for_work() {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return stop_ || failed_ || !q_.empty(); });
    return !failed_ && !q_.empty();
  }
  // FIFO admission under the lock: decide(front) is Take (popped into taken),
  // Hold (admission stops here) or Drop (popped into dropped, to be completed
  // by the caller with an error once the lock is released).
  template <class Decide>
  void admit(Decide&& decide, std::vector<T*>& taken, std::vector<T*>& dropped) {
    std::lock_guard<std::mutex> lk(mu_);
    while (!q_.empty() && !failed_) {
      T* r = q_.front();
      const Admit d = decide(r);
      if (d == Admit::Hold) break;
      q_.pop_front();
      (d == Admit::Take ? taken : dropped).push_back(r);
    }
  }
  // Stops accepting; the queued requests are still admitted.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
  }
  // Marks the server failed with a reason (the first reason is kept).
  void fail(const std::string& why) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (!failed_) err_ = why;
      failed_ = true;
    }
    cv_.notify_all();
  }
  bool failed() const {
    std::lock_guard<std::mutex> lk(mu_);
    return failed_;
  }
  std::string error() const {
    std::lock_guard<std::mutex> lk(mu_);
    return err_;
  }
  // Removes the first queued request for which match(r) holds and returns it
  // (the caller completes it), or NULL.
  template <class Match>
  T* remove_first(Match&& match) {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = q_.begin(); it != q_.end(); ++it)
      if (match(*it)) {
        T* r = *it;
        q_.erase(it);
        return r;
      }
    return nullptr;
  }
  // Removes and returns every queued request (the caller completes them).
  std::deque<T*> take_all() {
    std::lock_guard<std::mutex> lk(mu_);
    std::deque<T*> out;
    out.swap(q_);
    return out;
  }
  size_t size() const {
    std::lock_guard<std::mutex> lk(mu_);
    return q_.size();
  }

 private:
  mutable std::mutex mu_;
  std::condition_variable cv_;
  std::deque<T*> q_;
  size_t max_;
  bool stop_ = false, failed_ = false;
  std::string err_;
};

// One piece of a finished request's result: floats [begin, end) of the
// request's output, found at src + begin in a result buffer (`group`) that the
// requests finished by one tick share.  pending_req counts the request's
// pieces not yet copied, pending_group the group's.
template <class Req, class Group>
struct DeliveryPiece {
  Req* req = nullptr;
  const float* src = nullptr;
  float* dst = nullptr;
  size_t begin = 0, end = 0;
  Group* group = nullptr;
  std::shared_ptr<std::atomic<int>> pending_req, pending_group;
};

template <class Req, class Group>
class DeliveryQueue {
 public:
  using Piece = DeliveryPiece<Req, Group>;

  // Cuts the results of one group's requests into pieces of at most `chunk`
  // floats and queues them.  Each entry of reqs is (request, where its result
  // lies in the group's buffer, its output, its length in floats).
  void post(Group* group,
            const std::vector<std::tuple<Req*, const float*, float*, size_t>>& reqs,
            size_t chunk) {
    int pieces = 0;
    for (auto& r : reqs) pieces += (int)((std::get<3>(r) + chunk - 1) / chunk);
    auto pg = std::make_shared<std::atomic<int>>(pieces);
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (auto& r : reqs) {
        const size_t len = std::get<3>(r);
        auto pr = std::make_shared<std::atomic<int>>((int)((len + chunk - 1) / chunk));
        for (size_t b = 0; b < len; b += chunk) {
          Piece p;
          p.req = std::get<0>(r);
          p.src = std::get<1>(r);
          p.dst = std::get<2>(r);
          p.begin = b;
          p.end = b + chunk < len ? b + chunk : len;
          p.group = group;
          p.pending_req = pr;
          p.pending_group = pg;
          q_.push_back(std::move(p));
        }
      }
    }
    cv_.notify_all();
  }
  // Delivery thread: takes the next piece; false once stopped and empty.
  bool next(Piece& p) {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return stop_ || !q_.empty(); });
    if (q_.empty()) return false;
    p = std::move(q_.front());
    q_.pop_front();
    return true;
  }
  // Copies a piece to its client; calls req_done(req) after the request's
  // last piece and group_done(group) after the group's last piece.
  template <class ReqDone, class GroupDone>
  static void deliver(Piece& p, ReqDone&& req_done, GroupDone&& group_done) {
    std::memcpy(p.dst + p.begin, p.src + p.begin, (p.end - p.begin) * sizeof(float));
    if (p.pending_req->fetch_sub(1) == 1) req_done(p.req);
    if (p.pending_group->fetch_sub(1) == 1) group_done(p.group);
  }
  // Lets the delivery threads finish what is queued and return.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
  }

 private:
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Piece> q_;
  bool stop_ = false;
};

}  // namespace mg
