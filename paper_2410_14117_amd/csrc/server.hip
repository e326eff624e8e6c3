// server.hip -- continuous-batching serving loop for step/rollout requests of
// uneven env counts (the many-parallel-environments setting of Sec. II, served
// to many clients at once).
//
// Requests enter a FIFO admission queue.  A scheduler thread runs ticks: it
// admits queued requests while their pages fit under the memory cap, writes
// their envs into 64-env single-class pages (state + per-env factorisation,
// k_serve_join), advances every active page by one or more control steps with
// one launch over the pages of all classes (k_serve_tick), and retires
// finished requests (k_serve_leave gathers their states, one copy brings them
// to pinned host memory, a delivery thread copies them to the clients and
// frees the pages).  States stay on the device for the whole life of a
// request; requests that arrive while others run join at the next tick.  A
// tick's item arrays are written by the host into pinned memory that the
// kernels read through its device mapping, so a tick issues at most three
// launches and one copy.  A tick may advance each page by up to
// steps_per_tick control steps (as many as its request has left); the tick
// number is then a control-step clock that moves by steps_per_tick per tick.
#include "mg.h"
#include "mg_internal.h"
#include "page_pool.h"
#include "serve_book.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

using namespace mg;

namespace {

thread_local std::string g_server_create_error;

uint64_t clock_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket = 0;
  int64_t n = 0;
  int32_t L = 0, step = 0;
  std::vector<int32_t> cls;          // host copy of the env classes
  std::vector<int64_t> per_class;    // env count per class
  const float* x0 = nullptr;
  const float* mult = nullptr;
  const float* actions = nullptr;    // NULL: throttles generated from seed
  uint64_t seed = 0;
  int64_t ld = 0;
  float* out = nullptr;
  uint64_t arrival = 0;
  std::vector<int64_t> pages;
  std::vector<int32_t> page_cls;
  std::vector<int32_t> cols;         // [pages][64]
  std::vector<int32_t> entry;        // per page: its entry in the class's tick list
  int64_t t0 = 0;                    // tick of its first control step
  bool cancelled = false;            // retired without delivery (mg_server_cancel)
};

// Pinned host buffer mapped into the device's address space: the host writes
// it, kernels read or write it through `dev`.  It is allocated coherent
// (fine-grained), so the device neither caches stale copies of what the host
// rewrites for a later tick nor holds back what it writes for the host.
// Growth keeps the outgrown
// buffers until release(): freeing pinned memory can wait for the device,
// which would stall the tick pipeline, so the scheduler never frees;
// capacities double, so the retired buffers add up to less than the live one.
template <class T>
struct Pinned {
  T* h = nullptr;
  T* dev = nullptr;
  size_t cap = 0;
  std::vector<T*> outgrown;
  bool grow(size_t need) {
    if (need <= cap) return true;
    size_t c = std::max<size_t>(need, cap * 2 + 64);
    T *nh = nullptr, *nd = nullptr;
    if (hipHostMalloc((void**)&nh, c * sizeof(T), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void**)&nd, nh, 0) != hipSuccess || !nd) {
      (void)hipGetLastError();
      if (nh) (void)hipHostFree(nh);
      return false;
    }
    if (h) outgrown.push_back(h);
    h = nh;
    dev = nd;
    cap = c;
    return true;
  }
  void release() {
    if (h) outgrown.push_back(h);
    for (T* p : outgrown) (void)hipHostFree(p);
    outgrown.clear();
    h = nullptr;
    dev = nullptr;
    cap = 0;
  }
};

// Result buffer of a tick: device staging that the leave kernel gathers into
// and a pinned host buffer that one DMA copy fills (small scattered writes from
// the device straight into host memory measured several times slower).  The
// host side is pinned with the default flags: it is only ever read by the host
// after the copy has completed.  Growth keeps the outgrown pairs, as Pinned.
struct OutBuffer {
  float* h = nullptr;
  float* d = nullptr;
  size_t cap = 0;
  std::vector<std::pair<float*, float*>> outgrown;
  bool grow(size_t need) {
    if (need <= cap) return true;
    size_t c = std::max<size_t>(need, cap * 2 + 64);
    float *nh = nullptr, *nd = nullptr;
    if (hipHostMalloc((void**)&nh, c * sizeof(float), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&nd, c * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      if (nh) (void)hipHostFree(nh);
      return false;
    }
    if (h || d) outgrown.emplace_back(h, d);
    h = nh;
    d = nd;
    cap = c;
    return true;
  }
  void release() {
    if (h || d) outgrown.emplace_back(h, d);
    for (auto& hd : outgrown) {
      if (hd.first) (void)hipHostFree(hd.first);
      if (hd.second) (void)hipFree(hd.second);
    }
    outgrown.clear();
    h = nullptr;
    d = nullptr;
    cap = 0;
  }
};

}  // namespace

struct mg_server {
  int device = 0;
  int32_t D = 13, n_max = 1, substeps = 1, n_classes = 1;
  double dt = 0.005;
  bool fifo_plain = false;
  int32_t steps_per_tick = 1;        // most control steps a page advances per tick
  int64_t max_queue = 65536;
  // with a reservation, a tick joins at most stage_pages pages and retires at
  // most stage_pages pages and out_floats result floats (beyond a single
  // request); the rest waits a tick, so that serving allocates nothing
  bool reserved = false;
  size_t stage_pages = 0, out_floats = 0;
  std::vector<ClassConst> cc;
  std::vector<ClassNominal> nominal;
  ClassNominal* nominal_dev = nullptr;
  hipStream_t stream = nullptr;

  // pages
  int64_t page_floats = 0, slab_pages = 1024;
  std::unique_ptr<PagePool> pool;
  std::vector<float*> slab_blocks;
  std::vector<int32_t*> slab_cols;
  float* page_block(int64_t p) const {
    return slab_blocks[p / slab_pages] + (p % slab_pages) * page_floats;
  }
  int32_t* page_cols(int64_t p) const {
    return slab_cols[p / slab_pages] + (p % slab_pages) * kPageEnvs;
  }

  // ring of tick slots: each holds the staging buffers and event of one tick
  // in flight, so the host builds tick k+1 while the GPU runs tick k
  struct Slot {
    Pinned<ServeInitItem> init;       // pages joining in this tick
    Pinned<int32_t> cols_stage;       // their column maps
    Pinned<ServeGatherItem> gather;   // pages leaving after this tick
    OutBuffer* out = nullptr;     // pooled result buffer of this tick's finished requests
    hipEvent_t ev = nullptr;
    int64_t seq = 0;                  // 1-based number of the tick in this slot
    std::vector<Request*> retiring;   // finished by this tick, delivered on completion
  };
  // Finished requests' states sit in the pinned side of a tick's result buffer
  // that the tick's finished requests share; large results are cut into pieces
  // of kDeliverChunk floats that the delivery threads copy in parallel; a
  // request completes with its last piece, and the tick's last piece returns
  // the buffer to the pool.
  static constexpr size_t kDeliverChunk = (size_t)1 << 18;
  static constexpr int kDeliverThreads = 4;
  static constexpr int kSlots = 3;
  Slot slots[kSlots];
  std::deque<int> inflight;           // slot indices in issue order
  int next_slot = 0;
  int64_t tick_no = 0;                // control-step clock at the next tick's start

  // device-resident tick list: per class list_cap entries (a page's entry stays
  // put while its request runs); entries are reused lowest index first
  ServeTickItem* list_d = nullptr;
  size_t list_cap = 0;
  uint32_t* dbg_word = nullptr;       // the debug build's failed-check word, else NULL
  std::vector<std::set<int32_t>> free_entries;
  std::vector<int32_t> hw;            // per class: entries in use are below hw
  int32_t max_grid = 1024;            // blocks of the tick launch (4 pages each) at most
  ClassConst* cc_dev = nullptr;       // device copy of cc

  // admission queue (with the stop and failure state), tickets, thread
  std::unique_ptr<AdmissionQueue<Request>> queue;
  TicketBook book;
  std::mutex pool_mu;              // guards pool (scheduler admits, deliverers release)
  std::vector<Request*> active;    // scheduler thread only
  std::mutex err_mu;
  std::string err;                 // first failure, kept for mg_server_last_error
  int64_t fail_tick = 0;           // test hook: treat this tick's completion as failed
  // tickets of admitted requests to cancel at the next tick
  std::mutex cancel_mu;
  std::unordered_set<uint64_t> cancels;
  std::atomic<int64_t> n_cancels{0};
  std::thread thr;
  // delivery threads: copy finished requests' states to the clients, free their
  // pages and complete them, off the scheduler thread; a few of them, so that a
  // large result does not hold up the small ones finishing beside it
  std::thread deliver_thr[kDeliverThreads];
  DeliveryQueue<Request, OutBuffer> deliveries;
  std::mutex dmu;
  std::vector<OutBuffer*> out_pool;   // free pinned result buffers (guarded by dmu)
  std::vector<OutBuffer*> out_all;    // every result buffer, for teardown

  // statistics
  std::atomic<int64_t> completed{0}, rejected{0}, ticks{0}, env_steps{0}, active_envs{0},
      max_active_envs{0}, queued{0};
  std::atomic<int64_t> issue_ns{0}, wait_ns{0}, queue_ns{0}, max_queue_ns{0}, admitted_n{0};
  std::atomic<int64_t> max_issue_ns{0}, grow_events{0}, held_joins{0}, deferred_retires{0};
};

namespace {

// bounds of the debug build's checks in the serving kernels (scheduler thread)
DebugArgs serve_dbg(const mg_server* S) {
  DebugArgs d;
  d.word = S->dbg_word;
  d.cols = INT64_MAX;
  d.list = (int64_t)S->list_cap * S->n_classes;
  return d;
}

bool fail_server(mg_server* S, const std::string& msg) {
  {
    std::lock_guard<std::mutex> lk(S->err_mu);
    if (S->err.empty()) S->err = msg;
  }
  S->queue->fail(msg);
  return false;
}

#define SV_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return fail_server(S, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

ClassNominal class_nominal(const mg_vehicle& v) {
  ClassNominal n;
  std::memset(&n, 0, sizeof(n));
  n.p[0] = v.mass;
  for (int i = 0; i < 3; ++i) n.p[1 + i] = v.inertia[i];
  for (int i = 0; i < 6; ++i) {
    n.p[4 + i] = v.added_mass[i];
    n.p[10 + i] = v.d_lin[i];
    n.p[16 + i] = v.d_quad[i];
  }
  n.p[22] = v.buoyancy;
  n.zg = v.r_g[2];
  n.zb = v.r_b[2];
  n.n_thr = v.n_thr;
  n.lag = v.thr_tau > 0.0 ? 1 : 0;
  return n;
}

void finish(mg_server* S, Request* r, mg_status st) {
  if (st == MG_OK) S->completed.fetch_add(1);
  if (S->n_cancels.load() > 0) {
    std::lock_guard<std::mutex> lk(S->cancel_mu);
    if (S->cancels.erase(r->ticket)) S->n_cancels.store((int64_t)S->cancels.size());
  }
  S->book.close(r->ticket, st, clock_ns());
  delete r;
}

// A free result buffer from the pool; a new (empty) one if the pool is empty
// and allow_new, else NULL.
OutBuffer* take_out_buffer(mg_server* S, bool allow_new) {
  std::lock_guard<std::mutex> lk(S->dmu);
  if (!S->out_pool.empty()) {
    OutBuffer* m = S->out_pool.back();
    S->out_pool.pop_back();
    return m;
  }
  if (!allow_new) return nullptr;
  S->out_all.push_back(new OutBuffer());
  return S->out_all.back();
}

// Pinned / OutBuffer::grow, counting the growths that allocate (they cost host
// time in the scheduler; the counter shows whether a run was served from warm
// buffers).
template <class T>
bool grow_counted(mg_server* S, T& m, size_t need) {
  const size_t before = m.cap;
  const bool ok = m.grow(need);
  if (m.cap != before) S->grow_events.fetch_add(1);
  return ok;
}

// Grows the device tick list to hold `need` entries per class: waits for the
// stream and copies the host mirror into the new list.
bool grow_list(mg_server* S, size_t need, std::vector<ServeTickItem>& host) {
  size_t cap = std::max<size_t>(need, 2 * S->list_cap + 256);
  SV_HIP(hipStreamSynchronize(S->stream));
  std::vector<ServeTickItem> nh(cap * S->n_classes);
  std::memset(nh.data(), 0, nh.size() * sizeof(ServeTickItem));
  for (int c = 0; c < S->n_classes; ++c)
    for (size_t e = 0; e < S->list_cap; ++e) nh[c * cap + e] = host[c * S->list_cap + e];
  ServeTickItem* d = nullptr;
  SV_HIP(hipMalloc(&d, nh.size() * sizeof(ServeTickItem)));
  SV_HIP(hipMemcpy(d, nh.data(), nh.size() * sizeof(ServeTickItem), hipMemcpyHostToDevice));
  if (S->list_d) SV_HIP(hipFree(S->list_d));
  S->list_d = d;
  S->list_cap = cap;
  host.swap(nh);
  return true;
}

// Enqueue one tick into a free slot: initialise admitted pages and enter them
// in the tick list, advance every active page by up to steps_per_tick control
// steps, gather the states of the requests that finish into the slot's result
// buffer (copied to its pinned host side) and empty their list entries; record
// the slot's event.  Host
// work is proportional to the pages that join or leave, not to the pages in
// flight.
bool launch_tick(mg_server* S, mg_server::Slot& sl, std::vector<Request*>& admitted,
                 std::vector<ServeTickItem>& list_h) {
  // 1. newly admitted pages: list entries first (the list may grow), then one join launch
  size_t n_init = 0;
  for (Request* r : admitted) n_init += r->pages.size();
  if (n_init) {
    for (Request* r : admitted) {
      r->entry.resize(r->pages.size());
      for (size_t p = 0; p < r->pages.size(); ++p) {
        const int32_t c = r->page_cls[p];
        auto& fe = S->free_entries[c];
        int32_t e;
        if (!fe.empty()) {
          e = *fe.begin();
          fe.erase(fe.begin());
        } else {
          e = S->hw[c]++;
        }
        r->entry[p] = e;
      }
    }
    size_t need = 0;
    for (int c = 0; c < S->n_classes; ++c) need = std::max<size_t>(need, S->hw[c]);
    if (need > S->list_cap && !grow_list(S, need, list_h)) return false;
    if (!grow_counted(S, sl.init, n_init) || !grow_counted(S, sl.cols_stage, n_init * kPageEnvs))
      return fail_server(S, "pinned staging allocation failed");
    size_t k = 0;
    for (Request* r : admitted) {
      r->t0 = S->tick_no;
      for (size_t p = 0; p < r->pages.size(); ++p, ++k) {
        ServeInitItem& it = sl.init.h[k];
        std::memcpy(sl.cols_stage.h + k * kPageEnvs, r->cols.data() + p * kPageEnvs,
                    kPageEnvs * sizeof(int32_t));
        it.block = S->page_block(r->pages[p]);
        it.cols_src = sl.cols_stage.dev + k * kPageEnvs;
        it.cols = S->page_cols(r->pages[p]);
        it.x0 = r->x0;
        it.mult = r->mult;
        it.ld = r->ld;
        it.cls = r->page_cls[p];
        it.pad_ = 0;
        it.list_index = (int64_t)r->page_cls[p] * (int64_t)S->list_cap + r->entry[p];
        it.item.block = it.block;
        it.item.cols = it.cols;
        it.item.actions = r->actions;
        it.item.ld = r->ld;
        it.item.t0 = r->t0;
        it.item.L = r->L;
        it.item.pad_ = 0;
        it.item.seed = r->seed;
        it.item.n = r->n;
        list_h[it.list_index] = it.item;
      }
    }
    SV_HIP(launch_serve_join(sl.init.dev, (int32_t)n_init, S->list_d, S->nominal_dev, S->D,
                             serve_dbg(S), S->stream));
    for (Request* r : admitted) S->active.push_back(r);
    admitted.clear();
  }

  // cancelled requests retire this tick, without delivery (their pages still
  // run this tick's launch, to no effect on any other page)
  if (S->n_cancels.load() > 0) {
    std::lock_guard<std::mutex> lk(S->cancel_mu);
    for (Request* r : S->active)
      if (S->cancels.erase(r->ticket)) {
        r->cancelled = true;
        r->step = r->L;
      }
    S->n_cancels.store((int64_t)S->cancels.size());
  }

  // 2. the tick itself: every page advances min(K, steps its request has left);
  // the FIFO baseline runs S launches of one plain sub-step instead
  const int32_t K = S->steps_per_tick;
  int64_t envs = 0, env_steps = 0;
  for (Request* r : S->active) {
    envs += r->n;
    env_steps += r->n * std::min<int64_t>(K, r->L - r->step);
  }
  ServeTickArgs a;
  std::memset(&a, 0, sizeof(a));
  MG_SET_DBG(a, serve_dbg(S));
  a.list = S->list_d;
  a.cc = S->cc_dev;
  a.list_cap = (int64_t)S->list_cap;
  a.tick = S->tick_no;
  int64_t total = 0;
  for (int c = 0; c < S->n_classes; ++c) {
    a.count[c] = S->hw[c];
    total += S->hw[c];
  }
  a.n_classes = S->n_classes;
  a.steps = K;
  a.Dmax = S->D;
  a.n_max = S->n_max;
  a.substeps = S->fifo_plain ? 1 : S->substeps;
  a.dt = (float)S->dt;
  const int32_t grid = (int32_t)std::min<int64_t>(S->max_grid, std::max<int64_t>(1, (total + 3) / 4));
  const int reps = S->fifo_plain ? S->substeps : 1;
  for (int rep = 0; rep < reps; ++rep) SV_HIP(launch_serve_tick(a, grid, S->stream));
  S->active_envs.store(envs);
  if (envs > S->max_active_envs.load()) S->max_active_envs.store(envs);
  S->env_steps.fetch_add(env_steps);
  sl.seq = S->ticks.fetch_add(1) + 1;
  S->tick_no += K;

  // 3. the requests that have done their last control step retire, as many as
  // the reserved staging holds (always at least one); the others stay in the
  // tick list without work (their pages' step count is spent) until a later
  // tick has room
  std::vector<Request*> keep;
  size_t n_gat = 0, n_out = 0;
  for (Request* r : S->active) {
    r->step += (int32_t)std::min<int64_t>(K, r->L - r->step);
    if (r->step < r->L) {
      keep.push_back(r);
      continue;
    }
    const size_t g = r->pages.size(), o = (size_t)r->n * S->D;
    if (S->reserved && !sl.retiring.empty() &&
        (n_gat + g > S->stage_pages || n_out + o > S->out_floats)) {
      keep.push_back(r);
      S->deferred_retires.fetch_add(1);
      continue;
    }
    sl.retiring.push_back(r);
    n_gat += g;
    n_out += o;
  }
  if (!sl.retiring.empty()) {
    sl.out = take_out_buffer(S, !S->reserved);
    if (!sl.out) {
      // every reserved result buffer is still being delivered from
      S->deferred_retires.fetch_add((int64_t)sl.retiring.size());
      keep.insert(keep.end(), sl.retiring.begin(), sl.retiring.end());
      sl.retiring.clear();
      n_gat = n_out = 0;
    }
  }
  S->active.swap(keep);
  if (!sl.retiring.empty()) {
    if (!grow_counted(S, sl.gather, n_gat) || !grow_counted(S, *sl.out, n_out))
      return fail_server(S, "pinned result allocation failed");
    size_t k = 0, o = 0;
    for (Request* r : sl.retiring) {
      for (size_t p = 0; p < r->pages.size(); ++p, ++k) {
        ServeGatherItem& it = sl.gather.h[k];
        const int32_t c = r->page_cls[p];
        it.block = S->page_block(r->pages[p]);
        it.cols = S->page_cols(r->pages[p]);
        it.out = sl.out->d + o;
        it.n = r->n;
        it.list_index = (int64_t)c * (int64_t)S->list_cap + r->entry[p];
        std::memset(&list_h[it.list_index], 0, sizeof(ServeTickItem));
        S->free_entries[c].insert(r->entry[p]);
      }
      o += (size_t)r->n * S->D;
    }
    // the list shrinks from the top as its last entries empty
    for (int c = 0; c < S->n_classes; ++c) {
      auto& fe = S->free_entries[c];
      while (S->hw[c] > 0 && !fe.empty() && *fe.rbegin() == S->hw[c] - 1) {
        fe.erase(std::prev(fe.end()));
        --S->hw[c];
      }
    }
    SV_HIP(launch_serve_leave(sl.gather.dev, (int32_t)n_gat, S->list_d, S->D, serve_dbg(S),
                              S->stream));
    SV_HIP(hipMemcpyAsync(sl.out->h, sl.out->d, n_out * sizeof(float), hipMemcpyDeviceToHost,
                          S->stream));
  }
  SV_HIP(hipEventRecord(sl.ev, S->stream));
  return true;
}

// Completes the oldest tick in flight; `block` waits for it, otherwise only a
// finished one is taken.  Returns false on a device error.
bool retire_oldest(mg_server* S, bool block, bool* took) {
  *took = false;
  if (S->inflight.empty()) return true;
  mg_server::Slot& sl = S->slots[S->inflight.front()];
  const uint64_t t_wait = clock_ns();
  hipError_t e = block ? hipEventSynchronize(sl.ev) : hipEventQuery(sl.ev);
  if (block) S->wait_ns.fetch_add((int64_t)(clock_ns() - t_wait));
  if (e == hipErrorNotReady) return true;
  if (e == hipSuccess && sl.seq == S->fail_tick)
    return fail_server(S, "tick " + std::to_string(sl.seq) + ": failure injected by the host");
  if (e != hipSuccess) return fail_server(S, std::string("tick: ") + hipGetErrorString(e));
  S->inflight.pop_front();
  if (!sl.retiring.empty()) {
    std::vector<std::tuple<Request*, const float*, float*, size_t>> reqs;
    std::vector<Request*> cancelled;
    reqs.reserve(sl.retiring.size());
    size_t o = 0;
    for (Request* r : sl.retiring) {
      const size_t len = (size_t)r->n * S->D;
      if (r->cancelled)
        cancelled.push_back(r);
      else
        reqs.emplace_back(r, sl.out->h + o, r->out, len);
      o += len;
    }
    for (Request* r : cancelled) {
      {
        std::lock_guard<std::mutex> lk(S->pool_mu);
        S->pool->release(r->pages);
      }
      finish(S, r, MG_ERR_CANCELLED);
    }
    if (!reqs.empty()) {
      S->deliveries.post(sl.out, reqs, mg_server::kDeliverChunk);
    } else {
      std::lock_guard<std::mutex> lk(S->dmu);
      S->out_pool.push_back(sl.out);
    }
    sl.retiring.clear();
    sl.out = nullptr;
  }
  *took = true;
  return true;
}

// Copies pieces of finished requests to their clients; with a request's last
// piece frees its pages and completes it, with a tick's last piece returns
// the tick's result buffer to the pool.
void deliverer(mg_server* S) {
  DeliveryQueue<Request, OutBuffer>::Piece p;
  while (S->deliveries.next(p)) {
    DeliveryQueue<Request, OutBuffer>::deliver(
        p,
        [S](Request* r) {
          {
            std::lock_guard<std::mutex> lk(S->pool_mu);
            S->pool->release(r->pages);
          }
          finish(S, r, MG_OK);
        },
        [S](OutBuffer* o) {
          std::lock_guard<std::mutex> lk(S->dmu);
          S->out_pool.push_back(o);
        });
  }
}

void scheduler(mg_server* S) {
  (void)hipSetDevice(S->device);
  std::vector<Request*> admitted;
  std::vector<ServeTickItem> list_h(S->list_cap * S->n_classes);
  std::memset(list_h.data(), 0, list_h.size() * sizeof(ServeTickItem));
  bool ok = true;
  for (;;) {
    // deliver every tick the GPU has finished
    bool took = true;
    while (ok && took) ok = retire_oldest(S, false, &took);
    if (!ok) break;
    if (S->active.empty() && S->inflight.empty() && !S->queue->wait_for_work()) break;
    // FIFO admission while the pages fit under the cap (FIFO baseline: one request
    // at a time, the next admitted only once the previous one is delivered)
    using Admit = AdmissionQueue<Request>::Admit;
    std::vector<Request*> dropped;
    int64_t join_pages = 0;
    for (Request* r : admitted) join_pages += (int64_t)r->pages.size();
    S->queue->admit(
        [&](Request* r) {
          const bool busy = !S->active.empty() || !admitted.empty() || !S->inflight.empty();
          if (S->fifo_plain && busy) return Admit::Hold;
          const int64_t need = PagePool::pages_for(r->per_class);
          // a reserved server joins at most its staging's pages per tick
          if (S->reserved && !admitted.empty() && join_pages + need > (int64_t)S->stage_pages) {
            S->held_joins.fetch_add(1);
            return Admit::Hold;
          }
          std::vector<int64_t> pages;
          {
            std::lock_guard<std::mutex> lk(S->pool_mu);
            if (!S->pool->fits(need)) return Admit::Hold;
            if (!S->pool->allocate(need, pages)) {
              // the cap allows it but device memory could not be obtained: with
              // nothing in flight to free pages, this request cannot make progress
              if (busy) return Admit::Hold;
              S->queued.fetch_sub(1);
              return Admit::Drop;
            }
          }
          S->queued.fetch_sub(1);
          const int64_t qw = (int64_t)(clock_ns() - r->arrival);
          S->queue_ns.fetch_add(qw);
          S->admitted_n.fetch_add(1);
          if (qw > S->max_queue_ns.load()) S->max_queue_ns.store(qw);
          r->pages = pages;
          join_pages += need;
          return Admit::Take;
        },
        admitted, dropped);
    for (Request* r : dropped) finish(S, r, MG_ERR_OOM);
    if (S->queue->failed()) break;
    if (admitted.empty() && S->active.empty()) {
      // nothing to issue: wait for the oldest tick in flight (if any)
      if (!S->inflight.empty()) ok = retire_oldest(S, true, &took);
      if (!ok) break;
      continue;
    }
    // a free slot: the ring's oldest tick must have completed
    if ((int)S->inflight.size() == mg_server::kSlots) {
      ok = retire_oldest(S, true, &took);
      if (!ok) break;
    }
    const int k = S->next_slot;
    S->next_slot = (S->next_slot + 1) % mg_server::kSlots;
    const uint64_t t_issue = clock_ns();
    if (!launch_tick(S, S->slots[k], admitted, list_h)) break;
    const int64_t dt_issue = (int64_t)(clock_ns() - t_issue);
    S->issue_ns.fetch_add(dt_issue);
    if (dt_issue > S->max_issue_ns.load()) S->max_issue_ns.store(dt_issue);
    S->inflight.push_back(k);
  }
  // drain: anything left fails (device error or shutdown)
  if (!S->queue->failed()) {
    bool took = true;
    while (!S->inflight.empty() && took && retire_oldest(S, true, &took)) {
    }
  }
  const mg_status st = S->queue->failed() ? MG_ERR_DEVICE : MG_ERR_BUSY;
  S->deliveries.stop();
  for (auto& t : S->deliver_thr)
    if (t.joinable()) t.join();
  for (int k : S->inflight) {
    for (Request* r : S->slots[k].retiring) finish(S, r, st);
    S->slots[k].retiring.clear();
  }
  S->inflight.clear();
  for (Request* r : admitted) finish(S, r, st);
  for (Request* r : S->active) finish(S, r, st);
  S->active.clear();
  for (Request* r : S->queue->take_all()) {
    S->queued.fetch_sub(1);
    finish(S, r, st);
  }
}

}  // namespace

extern "C" {

uint64_t mg_clock_ns(void) { return clock_ns(); }

const char* mg_server_last_error(const mg_server* S) {
  if (!S) return g_server_create_error.c_str();
  std::lock_guard<std::mutex> lk(const_cast<mg_server*>(S)->err_mu);
  return S->err.c_str();
}

mg_status mg_server_create(const mg_server_config* cfg, mg_server** out) {
  auto bad = [](mg_status st, const char* m) {
    g_server_create_error = m;
    return st;
  };
  if (!out) return bad(MG_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg || cfg->abi_version != MG_ABI_VERSION) return bad(MG_ERR_INVALID, "bad config / ABI version");
  if (cfg->n_classes < 1 || cfg->n_classes > MG_MAX_CLASSES || !cfg->classes)
    return bad(MG_ERR_INVALID, "n_classes outside 1..16 or classes NULL");
  if (!(cfg->dt_sub > 0.0) || cfg->substeps < 1) return bad(MG_ERR_INVALID, "dt_sub / substeps");
  if (cfg->reserve_bytes < 0) return bad(MG_ERR_INVALID, "reserve_bytes < 0");
  if (cfg->steps_per_tick < 0 || cfg->steps_per_tick > 64)
    return bad(MG_ERR_INVALID, "steps_per_tick outside 0..64");
  if (cfg->fifo_plain && cfg->steps_per_tick > 1)
    return bad(MG_ERR_INVALID, "the FIFO plain baseline takes one control step per tick");
  for (int k = 0; k < cfg->n_classes; ++k) {
    const mg_vehicle& v = cfg->classes[k];
    if (v.n_thr < 1 || v.n_thr > MG_MAX_THRUSTERS || (v.thr_map != 0 && v.thr_map != 1) ||
        v.thr_tau < 0.0)
      return bad(MG_ERR_INVALID, "invalid vehicle class");
    if (v.r_g[0] != 0.0 || v.r_g[1] != 0.0 || v.r_b[0] != 0.0 || v.r_b[1] != 0.0)
      return bad(MG_ERR_UNSUPPORTED, "the GPU path needs r_g and r_b on the body z axis");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return bad(MG_ERR_DEVICE, "no HIP device");
  }
  if (cfg->device < 0 || cfg->device >= ndev) return bad(MG_ERR_INVALID, "bad device ordinal");
  if (hipSetDevice(cfg->device) != hipSuccess) return bad(MG_ERR_DEVICE, "hipSetDevice failed");

  auto S = std::make_unique<mg_server>();
  S->device = cfg->device;
  S->n_classes = cfg->n_classes;
  S->substeps = cfg->substeps;
  S->dt = cfg->dt_sub;
  S->fifo_plain = cfg->fifo_plain != 0;
  S->steps_per_tick = cfg->steps_per_tick > 1 ? cfg->steps_per_tick : 1;
  S->max_queue = cfg->max_queue > 0 ? cfg->max_queue : 65536;
  S->queue = std::make_unique<AdmissionQueue<Request>>((size_t)S->max_queue);
  if (const char* ft = std::getenv("MG_SERVER_FAIL_TICK")) S->fail_tick = std::atoll(ft);
  for (int k = 0; k < cfg->n_classes; ++k) {
    const mg_vehicle& v = cfg->classes[k];
    S->cc.push_back(make_class_const(v, cfg->dt_sub, cfg->substeps));
    S->nominal.push_back(class_nominal(v));
    S->n_max = std::max(S->n_max, v.n_thr);
    if (v.thr_tau > 0.0) S->D = std::max(S->D, 13 + v.n_thr);
  }
  S->page_floats = (int64_t)(S->D + kNumDerived) * kPageEnvs;
  const int64_t page_bytes = S->page_floats * 4 + kPageEnvs * 4;
  int64_t cap_bytes = cfg->mem_cap_bytes;
  if (cap_bytes <= 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return bad(MG_ERR_DEVICE, "hipMemGetInfo failed");
    const double frac = cfg->mem_fraction > 0.0 ? cfg->mem_fraction : 0.8;
    cap_bytes = (int64_t)(frac * (double)total_b);
  }
  const int64_t cap_pages = cap_bytes / page_bytes;
  if (cap_pages < 1) return bad(MG_ERR_INVALID, "memory cap below one page");
  S->slab_pages = std::min<int64_t>(1024, cap_pages);
  mg_server* raw = S.get();
  S->pool = std::make_unique<PagePool>(cap_pages, S->slab_pages, [raw](int64_t first, int64_t n) {
    (void)first;
    float* b = nullptr;
    int32_t* c = nullptr;
    if (hipMalloc((void**)&b, (size_t)n * raw->page_floats * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&c, (size_t)n * kPageEnvs * sizeof(int32_t)) != hipSuccess) {
      (void)hipGetLastError();
      if (b) (void)hipFree(b);
      return false;
    }
    raw->slab_blocks.push_back(b);
    raw->slab_cols.push_back(c);
    return true;
  });
  if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc(&S->nominal_dev, sizeof(ClassNominal) * S->n_classes) != hipSuccess ||
      hipMemcpy(S->nominal_dev, S->nominal.data(), sizeof(ClassNominal) * S->n_classes,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMalloc(&S->cc_dev, sizeof(ClassConst) * S->n_classes) != hipSuccess ||
      hipMemcpy(S->cc_dev, S->cc.data(), sizeof(ClassConst) * S->n_classes,
                hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    mg_server_destroy(S.release());
    return bad(MG_ERR_DEVICE, "server initialisation failed");
  }
  S->free_entries.resize(S->n_classes);
  S->hw.assign(S->n_classes, 0);
  // tick-list entries per class (64 envs each); grows by doubling, so a
  // reservation sizes it for every reserved page
  S->list_cap = (size_t)std::max<int64_t>(
      8192, std::min<int64_t>(cap_pages, std::max<int64_t>(0, cfg->reserve_bytes) / page_bytes));
#ifdef MG_DEBUG
  if (hipMalloc(&S->dbg_word, sizeof(uint32_t)) != hipSuccess ||
      hipMemset(S->dbg_word, 0, sizeof(uint32_t)) != hipSuccess) {
    (void)hipGetLastError();
    mg_server_destroy(S.release());
    return bad(MG_ERR_OOM, "debug word allocation failed");
  }
#endif
  {
    std::vector<ServeTickItem> z(S->list_cap * S->n_classes);
    std::memset(z.data(), 0, z.size() * sizeof(ServeTickItem));
    if (hipMalloc(&S->list_d, z.size() * sizeof(ServeTickItem)) != hipSuccess ||
        hipMemcpy(S->list_d, z.data(), z.size() * sizeof(ServeTickItem),
                  hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      mg_server_destroy(S.release());
      return bad(MG_ERR_DEVICE, "tick list allocation failed");
    }
  }
  for (auto& sl : S->slots) {
    if (hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      mg_server_destroy(S.release());
      return bad(MG_ERR_DEVICE, "tick slot initialisation failed");
    }
  }
  if (cfg->reserve_bytes > 0) {
    // pages up front, and staging for up to 4096 pages joining or leaving per
    // tick, so that serving within the reservation allocates nothing
    bool ok = S->pool->reserve(cfg->reserve_bytes / page_bytes);
    const size_t items = (size_t)std::min<int64_t>(4096, S->pool->created_pages());
    for (auto& sl : S->slots)
      ok = ok && sl.init.grow(items) && sl.cols_stage.grow(items * kPageEnvs) &&
           sl.gather.grow(items);
    // result buffers: one per slot in flight plus those the delivery thread
    // still copies out of (large outputs arriving in bursts), 16 MB each
    const size_t out_floats = std::min<size_t>(items * kPageEnvs * (size_t)S->D, (size_t)1 << 22);
    for (int i = 0; ok && i < 16; ++i) {
      S->out_all.push_back(new OutBuffer());
      S->out_pool.push_back(S->out_all.back());
      ok = S->out_all.back()->grow(out_floats);
    }
    S->reserved = true;
    S->stage_pages = items;
    S->out_floats = out_floats;
    if (!ok) {
      mg_server_destroy(S.release());
      return bad(MG_ERR_OOM, "could not reserve the requested page memory and staging");
    }
  }
  for (auto& t : S->deliver_thr) t = std::thread(deliverer, S.get());
  S->thr = std::thread(scheduler, S.get());
  *out = S.release();
  return MG_OK;
}

// Page layout of a request (independent of which pages it gets): pages per class
// in class order, each page's lanes take that class's envs in request order.
static void layout_pages(Request* r, int n_classes) {
  r->page_cls.clear();
  r->cols.assign((size_t)PagePool::pages_for(r->per_class) * kPageEnvs, -1);
  size_t p = 0;
  for (int c = 0; c < n_classes; ++c) {
    if (r->per_class[c] == 0) continue;
    int lane = 0;
    r->page_cls.push_back(c);
    for (int64_t e = 0; e < r->n; ++e) {
      if (r->cls[e] != c) continue;
      if (lane == kPageEnvs) {
        lane = 0;
        ++p;
        r->page_cls.push_back(c);
      }
      r->cols[p * kPageEnvs + lane++] = (int32_t)e;
    }
    ++p;
  }
}

mg_status mg_server_submit(mg_server* S, const mg_request* req, uint64_t* ticket) {
  if (!S || !req || !ticket) return MG_ERR_INVALID;
  if (req->n_envs < 1 || req->n_steps < 1 || !req->x0 || !req->out || req->ld < req->n_envs ||
      (req->actions_from_seed != 0 && req->actions_from_seed != 1) ||
      (!req->actions_from_seed && !req->actions))
    return MG_ERR_INVALID;
  auto r = std::make_unique<Request>();
  r->n = req->n_envs;
  r->L = req->n_steps;
  r->cls.assign(req->n_envs, 0);
  if (req->env_class) std::memcpy(r->cls.data(), req->env_class, sizeof(int32_t) * req->n_envs);
  r->per_class.assign(S->n_classes, 0);
  for (int32_t c : r->cls) {
    if (c < 0 || c >= S->n_classes) return MG_ERR_INVALID;
    ++r->per_class[c];
  }
  r->x0 = req->x0;
  r->mult = req->param_mult;
  r->actions = req->actions_from_seed ? nullptr : req->actions;
  r->seed = req->action_seed;
  r->ld = req->ld;
  r->out = req->out;
  // an arrival stamp in the future (a client submitting early) counts from submission
  const uint64_t now = clock_ns();
  r->arrival = (req->arrival_ns && req->arrival_ns < now) ? req->arrival_ns : now;
  // the cap is fixed at creation, so this test needs no lock
  const int64_t need = PagePool::pages_for(r->per_class);
  if (!S->pool->ever_fits(need)) {
    if (S->queue->failed()) return MG_ERR_DEVICE;
    S->rejected.fetch_add(1);
    return MG_ERR_INVALID;
  }
  layout_pages(r.get(), S->n_classes);
  Request* raw = r.get();
  const mg_status st = S->queue->push(raw, [&](Request* q) {
    q->ticket = S->book.open(q->arrival);
    S->queued.fetch_add(1);
  });
  if (st != MG_OK) return st;
  r.release();
  *ticket = raw->ticket;
  return MG_OK;
}

mg_status mg_server_cancel(mg_server* S, uint64_t ticket) {
  if (!S || !S->book.open_ticket(ticket)) return MG_ERR_INVALID;
  Request* r = S->queue->remove_first([&](Request* q) { return q->ticket == ticket; });
  if (r) {
    S->queued.fetch_sub(1);
    finish(S, r, MG_ERR_CANCELLED);
    return MG_OK;
  }
  // admitted (or about to be): the scheduler retires it at its next tick
  {
    std::lock_guard<std::mutex> lk(S->cancel_mu);
    S->cancels.insert(ticket);
    S->n_cancels.store((int64_t)S->cancels.size());
  }
  // it may have completed meanwhile: then the entry is dropped here
  if (!S->book.open_ticket(ticket)) {
    std::lock_guard<std::mutex> lk(S->cancel_mu);
    S->cancels.erase(ticket);
    S->n_cancels.store((int64_t)S->cancels.size());
  }
  return MG_OK;
}

mg_status mg_server_wait(mg_server* S, uint64_t ticket, int64_t timeout_us, double* latency_s) {
  if (!S) return MG_ERR_INVALID;
  return S->book.wait(ticket, timeout_us, latency_s);
}

mg_status mg_server_debug_word(mg_server* S, uint32_t* word, int32_t clear) {
  if (!S || !word) return MG_ERR_INVALID;
  *word = 0;
  if (!S->dbg_word) return MG_OK;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != S->device) (void)hipSetDevice(S->device);
  const bool ok =
      hipMemcpy(word, S->dbg_word, sizeof(uint32_t), hipMemcpyDeviceToHost) == hipSuccess &&
      (!clear || hipMemset(S->dbg_word, 0, sizeof(uint32_t)) == hipSuccess);
  if (!ok) (void)hipGetLastError();
  if (prev >= 0 && prev != S->device) (void)hipSetDevice(prev);
  return ok ? MG_OK : MG_ERR_DEVICE;
}

mg_status mg_server_get_stats(const mg_server* S, mg_server_stats* out) {
  if (!S || !out) return MG_ERR_INVALID;
  out->completed = S->completed.load();
  out->rejected = S->rejected.load();
  out->ticks = S->ticks.load();
  out->env_steps = S->env_steps.load();
  out->active_envs = S->active_envs.load();
  out->max_active_envs = S->max_active_envs.load();
  out->queued = S->queued.load();
  out->cap_pages = S->pool ? S->pool->cap_pages() : 0;
  out->created_pages = S->pool ? S->pool->created_pages() : 0;
  out->issue_ns = S->issue_ns.load();
  out->wait_ns = S->wait_ns.load();
  const int64_t na = S->admitted_n.load();
  out->mean_queue_ns = na ? S->queue_ns.load() / na : 0;
  out->max_queue_ns = S->max_queue_ns.load();
  out->max_issue_ns = S->max_issue_ns.load();
  out->grow_events = S->grow_events.load();
  out->held_joins = S->held_joins.load();
  out->deferred_retires = S->deferred_retires.load();
  return S->queue && S->queue->failed() ? MG_ERR_DEVICE : MG_OK;
}

void mg_server_destroy(mg_server* S) {
  if (!S) return;
  if (S->queue) S->queue->stop();
  if (S->thr.joinable()) S->thr.join();
  S->deliveries.stop();
  for (auto& t : S->deliver_thr)
    if (t.joinable()) t.join();
  (void)hipSetDevice(S->device);
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  for (auto& sl : S->slots) {
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    sl.init.release();
    sl.cols_stage.release();
    sl.gather.release();
  }
  for (OutBuffer* m : S->out_all) {
    m->release();
    delete m;
  }
  if (S->list_d) (void)hipFree(S->list_d);
  if (S->dbg_word) (void)hipFree(S->dbg_word);
  for (float* b : S->slab_blocks) (void)hipFree(b);
  for (int32_t* c : S->slab_cols) (void)hipFree(c);
  if (S->nominal_dev) (void)hipFree(S->nominal_dev);
  if (S->cc_dev) (void)hipFree(S->cc_dev);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  (void)hipGetLastError();
  delete S;
}

}  // extern "C"
