// Host-only concurrency check of the serving loop's bookkeeping (serve_book.h):
// many client threads submit into the bounded admission queue and wait on
// their tickets while a scheduler thread admits requests against a page cap,
// "runs" ticks that fill a shared result buffer, and posts the results in
// small pieces to four delivery threads that copy them out, free the pages and
// complete the tickets.  Extra waiters race the owners of some tickets.  A
// second run fails the server part-way.  Built with g++ -fsanitize=thread (the
// test also builds it with address,undefined); no GPU involved.  Prints the
// failures found and "N failures".
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "serve_book.h"

using namespace mg;

static std::atomic<int> failures{0};
#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      std::printf("FAIL line %d: %s\n", __LINE__, #c);                 \
      failures.fetch_add(1);                                           \
    }                                                                  \
  } while (0)

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Req {
  uint64_t ticket = 0, arrival = 0;
  int64_t pages = 0;
  float* out = nullptr;
  size_t len = 0;
};

struct Group {
  std::vector<float> data;
};

float value(uint64_t ticket, size_t i) { return (float)(ticket * 1000 + i % 997); }

constexpr int64_t kCap = 40;      // pages
constexpr size_t kChunk = 7;      // floats per delivered piece

struct Server {
  TicketBook book;
  AdmissionQueue<Req> queue{24};
  DeliveryQueue<Req, Group> deliveries;
  std::mutex pool_mu;
  int64_t free_pages = kCap;
  std::mutex gmu;
  std::vector<Group*> groups_free, groups_all;
  std::atomic<int64_t> completed{0};
  int fail_after_ticks = -1;      // < 0: never

  void finish(Req* r, mg_status st) {
    if (st == MG_OK) completed.fetch_add(1);
    book.close(r->ticket, st, now_ns());
    delete r;
  }

  void deliverer() {
    DeliveryQueue<Req, Group>::Piece p;
    while (deliveries.next(p)) {
      DeliveryQueue<Req, Group>::deliver(
          p,
          [this](Req* r) {
            {
              std::lock_guard<std::mutex> lk(pool_mu);
              free_pages += r->pages;
            }
            finish(r, MG_OK);
          },
          [this](Group* g) {
            std::lock_guard<std::mutex> lk(gmu);
            groups_free.push_back(g);
          });
    }
  }

  Group* take_group() {
    std::lock_guard<std::mutex> lk(gmu);
    if (!groups_free.empty()) {
      Group* g = groups_free.back();
      groups_free.pop_back();
      return g;
    }
    groups_all.push_back(new Group());
    return groups_all.back();
  }

  void scheduler() {
    using Admit = AdmissionQueue<Req>::Admit;
    int ticks = 0;
    for (;;) {
      if (!queue.wait_for_work()) break;
      std::vector<Req*> taken, dropped;
      queue.admit(
          [&](Req* r) {
            if (r->pages > kCap) return Admit::Drop;   // never fits
            std::lock_guard<std::mutex> lk(pool_mu);
            if (r->pages > free_pages) return Admit::Hold;
            free_pages -= r->pages;
            return Admit::Take;
          },
          taken, dropped);
      for (Req* r : dropped) finish(r, MG_ERR_OOM);
      if (taken.empty()) {
        std::this_thread::yield();   // pages come back from the delivery threads
        continue;
      }
      if (fail_after_ticks >= 0 && ticks == fail_after_ticks) {
        queue.fail("injected");
        for (Req* r : taken) finish(r, MG_ERR_DEVICE);
        break;
      }
      ++ticks;
      // one "tick": the results of the admitted requests back to back in a group
      Group* g = take_group();
      size_t total = 0;
      for (Req* r : taken) total += r->len;
      g->data.resize(total);
      std::vector<std::tuple<Req*, const float*, float*, size_t>> reqs;
      size_t o = 0;
      for (Req* r : taken) {
        for (size_t i = 0; i < r->len; ++i) g->data[o + i] = value(r->ticket, i);
        reqs.emplace_back(r, g->data.data() + o, r->out, r->len);
        o += r->len;
      }
      deliveries.post(g, reqs, kChunk);
    }
    const mg_status st = queue.failed() ? MG_ERR_DEVICE : MG_ERR_BUSY;
    for (Req* r : queue.take_all()) finish(r, st);
  }
};

struct Sub {
  uint64_t ticket = 0;
  size_t len;
  int64_t pages;
  std::vector<float> out;
};

// n_clients threads submit n_req requests each, retrying while the queue is
// full, then wait on every ticket; `racers` more threads wait on client 0's
// tickets at the same time.  With fail_after >= 0 the scheduler fails the
// server after that many ticks.
void run(int n_clients, int n_req, int racers, int fail_after) {
  Server S;
  S.fail_after_ticks = fail_after;
  std::thread sched([&] { S.scheduler(); });
  std::thread del[4];
  for (auto& t : del) t = std::thread([&] { S.deliverer(); });

  std::vector<std::vector<Sub>> subs(n_clients);
  std::atomic<bool> client0_submitted{false};
  std::vector<std::atomic<int>> ok_count(n_req);
  for (auto& c : ok_count) c.store(0);
  std::atomic<int64_t> ok_total{0}, dev_total{0}, oom_total{0}, refused_dev{0};

  auto check_result = [&](Sub& s, mg_status st, double lat) {
    if (st == MG_OK) {
      ok_total.fetch_add(1);
      CHECK(s.pages <= kCap);
      CHECK(lat >= 0.0);
      for (size_t i = 0; i < s.len; ++i)
        if (s.out[i] != value(s.ticket, i)) {
          CHECK(s.out[i] == value(s.ticket, i));
          break;
        }
    } else if (st == MG_ERR_OOM) {
      oom_total.fetch_add(1);
      CHECK(s.pages > kCap);
    } else {
      CHECK(st == MG_ERR_DEVICE && fail_after >= 0);
      dev_total.fetch_add(1);
    }
  };

  std::vector<std::thread> clients;
  for (int c = 0; c < n_clients; ++c)
    clients.emplace_back([&, c] {
      std::mt19937_64 g(1234 + c);
      auto& mine = subs[c];
      mine.reserve(n_req);
      for (int k = 0; k < n_req; ++k) {
        Sub s;
        s.len = 1 + g() % 40;
        s.pages = (g() % 50 == 0) ? kCap + 1 : 1 + (int64_t)(g() % 6);
        s.out.assign(s.len, -1.0f);
        mine.push_back(std::move(s));
        Sub& m = mine.back();
        auto* r = new Req();
        r->pages = m.pages;
        r->out = m.out.data();
        r->len = m.len;
        r->arrival = now_ns();
        mg_status st;
        // the ticket is read inside the push: once queued, r belongs to the server
        // and may be completed and freed at any moment
        while ((st = S.queue.push(r, [&](Req* q) {
                  q->ticket = S.book.open(q->arrival);
                  m.ticket = q->ticket;
                })) == MG_ERR_BUSY)
          std::this_thread::yield();
        if (st != MG_OK) {
          CHECK(st == MG_ERR_DEVICE && fail_after >= 0);
          refused_dev.fetch_add(1);
          delete r;
          mine.pop_back();
          continue;
        }
      }
      if (c == 0) client0_submitted.store(true);
      for (size_t k = 0; k < mine.size(); ++k) {
        double lat = -1;
        const mg_status st = S.book.wait(mine[k].ticket, -1, &lat);
        if (c == 0) {
          if (st == MG_ERR_INVALID) continue;   // a racer consumed it
          ok_count[k].fetch_add(1);
        }
        check_result(mine[k], st, lat);
      }
    });
  std::vector<std::thread> racer_thr;
  for (int r = 0; r < racers; ++r)
    racer_thr.emplace_back([&] {
      while (!client0_submitted.load()) std::this_thread::yield();
      auto& mine = subs[0];
      for (size_t k = 0; k < mine.size(); ++k) {
        double lat = -1;
        const mg_status st = S.book.wait(mine[k].ticket, -1, &lat);
        if (st == MG_ERR_INVALID) continue;   // the owner or another racer consumed it
        ok_count[k].fetch_add(1);
        check_result(mine[k], st, lat);
      }
    });
  for (auto& t : clients) t.join();
  for (auto& t : racer_thr) t.join();
  for (size_t k = 0; k < subs[0].size(); ++k) CHECK(ok_count[k].load() == 1);
  S.queue.stop();
  sched.join();
  S.deliveries.stop();
  for (auto& t : del) t.join();
  int64_t submitted = 0;
  for (auto& v : subs) submitted += (int64_t)v.size();
  CHECK(ok_total.load() + dev_total.load() + oom_total.load() == submitted);
  CHECK(S.book.size() == 0);
  CHECK(S.queue.size() == 0);
  if (fail_after < 0) {
    CHECK(dev_total.load() == 0 && refused_dev.load() == 0);
    CHECK(S.free_pages == kCap);
    CHECK(S.completed.load() == ok_total.load());
  } else {
    CHECK(dev_total.load() + refused_dev.load() > 0);
  }
  for (Group* g : S.groups_all) delete g;
  std::printf("run clients=%d req=%d racers=%d fail_after=%d: ok %lld, device %lld, oom %lld, "
              "refused %lld\n",
              n_clients, n_req, racers, fail_after, (long long)ok_total.load(),
              (long long)dev_total.load(), (long long)oom_total.load(),
              (long long)refused_dev.load());
}

void single_thread_cases() {
  TicketBook b;
  const uint64_t t = b.open(100);
  double lat = -1;
  CHECK(b.open_ticket(t) && !b.open_ticket(t + 1));
  CHECK(b.wait(t, 1000, &lat) == MG_ERR_BUSY);          // not completed: times out
  CHECK(b.wait(t + 1, 0, &lat) == MG_ERR_INVALID);      // never issued
  b.close(t, MG_OK, 600);
  CHECK(!b.open_ticket(t));
  b.close(t, MG_ERR_DEVICE, 900);                       // a second close is ignored
  CHECK(b.wait(t, -1, &lat) == MG_OK && std::fabs(lat - 500e-9) < 1e-15);
  CHECK(b.wait(t, -1, &lat) == MG_ERR_INVALID);         // consumed
  CHECK(b.size() == 0);
  AdmissionQueue<Req> q(2);
  Req a, c, d;
  auto none = [](Req*) {};
  CHECK(q.push(&a, none) == MG_OK && q.push(&c, none) == MG_OK);
  CHECK(q.push(&d, none) == MG_ERR_BUSY);               // full
  CHECK(q.remove_first([&](Req* r) { return r == &c; }) == &c && q.size() == 1);
  CHECK(q.remove_first([&](Req* r) { return r == &c; }) == nullptr);
  CHECK(q.push(&c, none) == MG_OK && q.size() == 2);
  std::vector<Req*> taken, dropped;
  int seen = 0;
  q.admit([&](Req*) { return ++seen == 1 ? AdmissionQueue<Req>::Admit::Take
                                         : AdmissionQueue<Req>::Admit::Hold; },
          taken, dropped);
  CHECK(taken.size() == 1 && taken[0] == &a && dropped.empty() && q.size() == 1);
  q.fail("x");
  q.fail("y");
  CHECK(q.failed() && q.error() == "x");
  CHECK(q.push(&d, none) == MG_ERR_DEVICE);
  CHECK(!q.wait_for_work());
  CHECK(q.take_all().size() == 1);
}

}  // namespace

int main() {
  single_thread_cases();
  run(16, 300, 3, -1);
  run(16, 300, 2, 25);
  run(4, 50, 1, 0);
  std::printf("%d failures\n", failures.load());
  return failures.load() ? 1 : 0;
}
