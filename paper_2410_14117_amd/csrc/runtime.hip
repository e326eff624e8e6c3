// runtime.hip -- host side of libmg: the sim context (SoA device buffers,
// class-grouped env layout, per-class constants), argument checking, launch
// sequencing, HIP-graph cache and the exported C ABI of include/mg.h.
#include "mg.h"
#include "mg_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace mg;

// Recomputation scratch of mg_adj_backward_noalloc: one copy per device,
// allocated when the library's device code is loaded and held until the
// process ends.  Host code never uses this name as an address (on the host it
// is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns, kept per device in g_noalloc_ptr.
static __device__ __align__(256) float scratch[MG_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace {

thread_local std::string g_create_error;

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
float* g_noalloc_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, looked up once per device with
// that device current (the caller's DeviceGuard makes it so); NULL if the
// lookup fails or the ordinal is beyond kMaxDevices.
float* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_noalloc_ptr[device] = static_cast<float*>(p);
  }
  return g_noalloc_ptr[device];
}

constexpr size_t kMaxCachedGraphs = 64;   // rollout graphs kept per sim

struct GraphKey {
  int32_t T, plain;
  const void *actions, *targets, *traj, *stats;
  bool operator<(const GraphKey& o) const {
    return std::tie(T, plain, actions, targets, traj, stats) <
           std::tie(o.T, o.plain, o.actions, o.targets, o.traj, o.stats);
  }
};

}  // namespace

struct mg_sim {
  int device = 0;
  int n_cu = 0;                      // compute units of the device
  hipStream_t stream = nullptr;      // caller's stream (not owned)
  hipStream_t cap_stream = nullptr;  // owned, used only to capture graphs
  // one helper stream per class after the first: the classes' launches are
  // independent, so they run as parallel chains (fork/join through events) and
  // one class's tail of blocks overlaps the other's
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> ev_fork, ev_join;
  bool broken = false;
  std::string err;

  int64_t E = 0, Ep = 0;
  int32_t D = 13, n_max = 1, substeps = 1, n_classes = 1;
  double dt = 0.01;
  int32_t nblk_total = 0;

  std::vector<ClassConst> cc;
  std::vector<ClassNominal> nominal;
  std::vector<int64_t> seg_start, seg_len;
  std::vector<int32_t> seg_blk_off;

  float* state = nullptr;      // [D][Ep]
  float* params = nullptr;     // [23][Ep]
  float* derived = nullptr;    // [kNumDerived][Ep]
  int32_t* perm = nullptr;     // [Ep] internal -> caller (-1 for padding), NULL = identity
  int32_t* iperm = nullptr;    // [E] caller -> internal, NULL = identity
  uint8_t* class_of = nullptr; // [Ep]
  uint8_t* flags = nullptr;    // [Ep] status flags (kFlagNonFinite, kFlagNotSPD)
  ClassNominal* nominal_dev = nullptr;
  double* partials = nullptr;
  size_t partials_cap = 0;     // doubles
  float* staging = nullptr;    // [max(D,23)][E] for host copies with a permuted layout
  float* segbuf = nullptr;     // adjoint recomputation scratch
  size_t segbuf_cap = 0;       // floats
  std::map<GraphKey, hipGraphExec_t> graphs;
  // Gym-style task (mg_task_configure)
  bool task_on = false;
  TaskConst task{};
  float* task_f = nullptr;     // [5][Ep] centre, curve phase, target yaw
  int32_t* task_k = nullptr;   // [Ep] control steps since each env's episode began
  // split scheme (mg_step_split): each env's acceleration of its last sub-step
  float* split_acc = nullptr;  // [6][Ep]
  // bounds checks of the debug build: the failed-check word (NULL in the
  // release build) and the bounds the kernels check against
  DebugArgs dbg{};
};

// Class constants the step kernels read from scalar registers.
ClassConst mg::make_class_const(const mg_vehicle& v, double dt, int substeps) {
  ClassConst c;
  std::memset(&c, 0, sizeof(c));
  for (int i = 0; i < v.n_thr; ++i) {
    const double* r = v.thr_pos[i];
    const double* d = v.thr_dir[i];
    const double col[6] = {d[0], d[1], d[2], r[1] * d[2] - r[2] * d[1],
                           r[2] * d[0] - r[0] * d[2], r[0] * d[1] - r[1] * d[0]};
    for (int k = 0; k < 6; ++k) c.B[k][i] = (float)col[k];
  }
  c.f_max = (float)v.f_max;
  c.inv_tau = v.thr_tau > 0.0 ? (float)(1.0 / v.thr_tau) : 0.0f;
  const double z = v.thr_tau > 0.0 ? dt / v.thr_tau : 0.0;
  const double rho = 1.0 - z + z * z / 2 - z * z * z / 6 + z * z * z * z / 24;
  c.sigma2 = (float)(1.0 - z / 2);
  c.sigma3 = (float)(1.0 - z / 2 + z * z / 4);
  c.sigma4 = (float)(1.0 - z + z * z / 2 - z * z * z / 4);
  c.rho = (float)rho;
  c.rho_s = (float)std::pow(rho, (double)substeps);
  c.n_thr = v.n_thr;
  c.thr_map = v.thr_map;
  c.lag = v.thr_tau > 0.0 ? 1 : 0;
  return c;
}

namespace {

mg_status fail(mg_sim* s, mg_status code, const std::string& msg) {
  if (s) {
    s->err = msg;
    if (code == MG_ERR_DEVICE) s->broken = true;
  } else {
    g_create_error = msg;
  }
  return code;
}

#define MG_HIP(sim, call)                                                               \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail((sim), MG_ERR_DEVICE,                                                 \
                  std::string(#call) + ": " + hipGetErrorString(e_));                   \
  } while (0)

// Makes the sim's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

mg_status check_usable(mg_sim* s) {
  if (!s) return MG_ERR_INVALID;
  if (s->broken) return MG_ERR_DEVICE;
  return MG_OK;
}

void clear_graphs(mg_sim* s) {
  for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
  s->graphs.clear();
}

ClassNominal make_nominal(const mg_vehicle& v) {
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

bool finite_all(const double* p, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

mg_status validate_vehicle(const mg_vehicle& v, int idx, std::string& why, bool& unsupported) {
  unsupported = false;
  char buf[160];
  if (v.n_thr < 1 || v.n_thr > MG_MAX_THRUSTERS) {
    std::snprintf(buf, sizeof buf, "class %d: n_thr %d outside 1..%d", idx, v.n_thr,
                  MG_MAX_THRUSTERS);
    why = buf;
    return MG_ERR_INVALID;
  }
  if (v.thr_map != 0 && v.thr_map != 1) {
    std::snprintf(buf, sizeof buf, "class %d: thr_map must be 0 or 1", idx);
    why = buf;
    return MG_ERR_INVALID;
  }
  const double scal[4] = {v.mass, v.buoyancy, v.f_max, v.thr_tau};
  if (!finite_all(scal, 4) || !finite_all(v.inertia, 3) || !finite_all(v.added_mass, 6) ||
      !finite_all(v.d_lin, 6) || !finite_all(v.d_quad, 6) || !finite_all(v.r_g, 3) ||
      !finite_all(v.r_b, 3) || !finite_all(&v.thr_pos[0][0], 3 * v.n_thr) ||
      !finite_all(&v.thr_dir[0][0], 3 * v.n_thr) || v.thr_tau < 0.0) {
    std::snprintf(buf, sizeof buf, "class %d: non-finite or negative lag parameter", idx);
    why = buf;
    return MG_ERR_INVALID;
  }
  if (v.r_g[0] != 0.0 || v.r_g[1] != 0.0 || v.r_b[0] != 0.0 || v.r_b[1] != 0.0) {
    std::snprintf(buf, sizeof buf,
                  "class %d: the GPU path needs r_g and r_b on the body z axis", idx);
    why = buf;
    unsupported = true;
    return MG_ERR_UNSUPPORTED;
  }
  return MG_OK;
}

mg_status ensure_partials(mg_sim* s, int32_t n_ctrl) {
  const size_t need = (size_t)std::max(n_ctrl, 1) * (size_t)s->nblk_total * 4;
  if (need <= s->partials_cap) return MG_OK;
  // a graph may hold the old buffer: drop the cache before freeing it
  MG_HIP(s, hipStreamSynchronize(s->stream));
  clear_graphs(s);
  if (s->partials) MG_HIP(s, hipFree(s->partials));
  s->partials = nullptr;
  s->partials_cap = 0;
  if (hipMalloc(&s->partials, need * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    s->partials = nullptr;
    return fail(s, MG_ERR_OOM, "partials allocation failed");
  }
  s->partials_cap = need;
  return MG_OK;
}

// Enqueue n_ctrl fused control steps (plain = 0) or their plain equivalent
// (one launch per sub-step), followed by the statistics pass.  Class k >= 1
// runs on helper stream k-1, forked from and joined back into `st`.
mg_status enqueue_steps(mg_sim* s, hipStream_t st, const float* actions, int32_t n_ctrl,
                        const float* targets, float* traj, double* stats, bool plain,
                        bool one_launch_per_ctrl) {
  StepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.state = s->state;
  a.flags = s->flags;
  MG_SET_DBG(a, s->dbg);
  a.derived = s->derived;
  a.Ep = s->Ep;
  a.E = s->E;
  a.perm = s->perm;
  a.n_max = s->n_max;
  a.targets = targets;
  a.D = s->D;
  a.nblk_total = s->nblk_total;
  a.dt = (float)s->dt;
  const int64_t frame = (int64_t)s->n_max * s->E;
  const int64_t tframe = (int64_t)s->D * s->E;
  const int64_t pframe = (int64_t)s->nblk_total * 4;
  for (int k = 1; k < s->n_classes; ++k) {
    MG_HIP(s, hipEventRecord(s->ev_fork[k - 1], st));
    MG_HIP(s, hipStreamWaitEvent(s->aux[k - 1], s->ev_fork[k - 1], 0));
  }
  for (int k = 0; k < s->n_classes; ++k) {
    hipStream_t ks = k == 0 ? st : s->aux[k - 1];
    a.seg_start = s->seg_start[k];
    a.seg_len = s->seg_len[k];
    a.blk_off = s->seg_blk_off[k];
    if (!plain && !one_launch_per_ctrl) {
      a.actions = actions;
      a.traj = traj;
      a.partials = stats ? s->partials : nullptr;
      a.n_ctrl = n_ctrl;
      a.substeps = s->substeps;
      MG_HIP(s, launch_step(s->cc[k], a, ks));
      continue;
    }
    const int32_t n_sub = plain ? s->substeps : 1;
    for (int32_t t = 0; t < n_ctrl; ++t) {
      for (int32_t sub = 0; sub < n_sub; ++sub) {
        const bool last = sub == n_sub - 1;
        a.actions = actions + t * frame;
        a.traj = (traj && last) ? traj + t * tframe : nullptr;
        a.partials = (stats && last) ? s->partials + t * pframe : nullptr;
        a.n_ctrl = 1;
        a.substeps = plain ? 1 : s->substeps;
        MG_HIP(s, launch_step(s->cc[k], a, ks));
      }
    }
  }
  for (int k = 1; k < s->n_classes; ++k) {
    MG_HIP(s, hipEventRecord(s->ev_join[k - 1], s->aux[k - 1]));
    MG_HIP(s, hipStreamWaitEvent(st, s->ev_join[k - 1], 0));
  }
  if (stats) MG_HIP(s, launch_stats_finalize(s->partials, s->nblk_total, n_ctrl, stats, st));
  return MG_OK;
}

mg_status reset_impl(mg_sim* s, const int64_t* ids, int64_t n, const float* state_in,
                     const float* param_in, int absolute, int write_state) {
  ResetArgs r;
  std::memset(&r, 0, sizeof(r));
  r.state = s->state;
  r.flags = s->flags;
  MG_SET_DBG(r, s->dbg);
  r.params = s->params;
  r.derived = s->derived;
  r.Ep = s->Ep;
  r.E = s->E;
  r.D = s->D;
  r.iperm = s->iperm;
  r.class_of = s->class_of;
  r.nominal = s->nominal_dev;
  r.ids = ids;
  r.n = n;
  r.state_in = state_in;
  r.param_in = param_in;
  r.param_absolute = absolute;
  r.write_state = write_state;
  r.task_k = s->task_k;
  r.split_acc = s->split_acc;
  MG_HIP(s, launch_reset(r, s->stream));
  return MG_OK;
}

// internal [rows][Ep] -> caller [rows][E] at out (device), or via staging to host
mg_status copy_out(mg_sim* s, const float* src, int32_t rows, float* out, int32_t on_device) {
  if (!out) return fail(s, MG_ERR_INVALID, "output pointer is NULL");
  float* dst = on_device ? out : s->staging;
  if (!s->perm) {
    MG_HIP(s, hipMemcpy2DAsync(dst, s->E * sizeof(float), src, s->Ep * sizeof(float),
                               s->E * sizeof(float), rows, hipMemcpyDeviceToDevice, s->stream));
  } else {
    MG_HIP(s, launch_gather_out(src, s->Ep, dst, s->E, rows, s->perm, s->Ep, s->stream));
  }
  if (!on_device) {
    MG_HIP(s, hipMemcpyAsync(out, s->staging, (size_t)rows * s->E * sizeof(float),
                             hipMemcpyDeviceToHost, s->stream));
    MG_HIP(s, hipStreamSynchronize(s->stream));
  }
  return MG_OK;
}

mg_status step_common(mg_sim* s, const float* actions, int32_t n_ctrl, const float* targets,
                      float* traj, double* stats, bool plain) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!actions) return fail(s, MG_ERR_INVALID, "actions is NULL");
  if (n_ctrl < 1) return fail(s, MG_ERR_INVALID, "n_ctrl must be >= 1");
  DeviceGuard g(s->device);
  if (stats && (st = ensure_partials(s, n_ctrl))) return st;
  return enqueue_steps(s, s->stream, actions, n_ctrl, targets, traj, stats, plain, false);
}

mg_status adj_common(mg_sim* s, const float* actions, int32_t T, int32_t K, const float* ckpt) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!actions || !ckpt) return fail(s, MG_ERR_INVALID, "actions and ckpt must not be NULL");
  if (T < 1 || K < 1) return fail(s, MG_ERR_INVALID, "T and ckpt_every must be >= 1");
  return MG_OK;
}

AdjArgs adj_args(mg_sim* s, const float* actions, int32_t T, int32_t K) {
  AdjArgs a;
  std::memset(&a, 0, sizeof(a));
  a.state = s->state;
  a.derived = s->derived;
  a.Ep = s->Ep;
  a.E = s->E;
  a.perm = s->perm;
  a.actions = actions;
  a.n_max = s->n_max;
  a.D = s->D;
  a.T = T;
  a.substeps = s->substeps;
  a.ckpt_every = K;
  a.dt = (float)s->dt;
  a.n_cu = s->n_cu;
  MG_SET_DBG(a, s->dbg);
  return a;
}

// Whether the backward reads its inputs from the forward's trajectory: the
// caller passed one, and each control step is a single sub-step.
bool traj_inputs(const mg_sim* s, const float* traj) {
  return traj && s->substeps == 1;
}

// The backward's launches: per class, the whole rollout's recomputation into
// buf (whole) and the reverse sweep, or the sweep that recomputes each segment
// into buf itself; with traj (one sub-step per control step) only the sweep,
// reading its inputs from traj.  Allocates nothing.
mg_status adj_backward_launch(mg_sim* s, const float* ckpt, const float* traj,
                              const float* actions, int32_t T, int32_t ckpt_every,
                              const float* dL_dtraj, float* dL_dact, float* dL_dtheta,
                              float* dL_dx0, float* buf, bool whole) {
  AdjArgs a = adj_args(s, actions, T, ckpt_every);
  a.ckpt = const_cast<float*>(ckpt);
  a.traj = const_cast<float*>(traj);
  a.gtraj = dL_dtraj;
  a.gact = dL_dact;
  a.gtheta = dL_dtheta;
  a.gx0 = dL_dx0;
  a.segbuf = buf;
  a.recomputed = traj ? 2 : (whole ? 1 : 0);
  for (int k = 0; k < s->n_classes; ++k) {
    a.seg_start = s->seg_start[k];
    a.seg_len = s->seg_len[k];
    a.zb = (float)s->nominal[k].zb;
    if (whole && !traj) MG_HIP(s, launch_adj_recompute(s->cc[k], a, s->stream));
    MG_HIP(s, launch_adjoint(true, s->cc[k], a, s->stream));
  }
  return MG_OK;
}

// internal [rows][Ep] <- caller [rows][E] (device)
mg_status copy_in(mg_sim* s, const float* src, int32_t rows, float* dst) {
  if (!s->perm) {
    MG_HIP(s, hipMemcpy2DAsync(dst, s->Ep * sizeof(float), src, s->E * sizeof(float),
                               s->E * sizeof(float), rows, hipMemcpyDeviceToDevice, s->stream));
  } else {
    MG_HIP(s, launch_scatter_in(src, s->E, dst, s->Ep, rows, s->perm, s->Ep, s->stream));
  }
  return MG_OK;
}

// One task launch per class (forked / joined like the step): a Gym step when
// actions is given, else the observation alone.
mg_status enqueue_task(mg_sim* s, const float* actions, float* obs, float* err, int32_t* done,
                       const float* reset_state, const float* reset_mult) {
  hipStream_t st = s->stream;
  TaskArgs a;
  std::memset(&a, 0, sizeof(a));
  a.state = s->state;
  a.flags = s->flags;
  MG_SET_DBG(a, s->dbg);
  a.params = s->params;
  a.derived = s->derived;
  a.task_f = s->task_f;
  a.task_k = s->task_k;
  a.Ep = s->Ep;
  a.E = s->E;
  a.perm = s->perm;
  a.actions = actions;
  a.n_max = s->n_max;
  a.D = s->D;
  a.substeps = s->substeps;
  a.dt = (float)s->dt;
  a.obs = obs;
  a.err = err;
  a.done = done;
  a.reset_state = reset_state;
  a.reset_mult = reset_mult;
  for (int k = 1; k < s->n_classes; ++k) {
    MG_HIP(s, hipEventRecord(s->ev_fork[k - 1], st));
    MG_HIP(s, hipStreamWaitEvent(s->aux[k - 1], s->ev_fork[k - 1], 0));
  }
  for (int k = 0; k < s->n_classes; ++k) {
    a.seg_start = s->seg_start[k];
    a.seg_len = s->seg_len[k];
    a.nominal = s->nominal_dev + k;
    MG_HIP(s, launch_task(s->cc[k], s->task, a, k == 0 ? st : s->aux[k - 1]));
  }
  for (int k = 1; k < s->n_classes; ++k) {
    MG_HIP(s, hipEventRecord(s->ev_join[k - 1], s->aux[k - 1]));
    MG_HIP(s, hipStreamWaitEvent(st, s->ev_join[k - 1], 0));
  }
  return MG_OK;
}

}  // namespace

extern "C" {

uint32_t mg_abi_version(void) { return MG_ABI_VERSION; }

const char* mg_status_str(mg_status s) {
  switch (s) {
    case MG_OK: return "ok";
    case MG_ERR_INVALID: return "invalid argument";
    case MG_ERR_OOM: return "out of device memory";
    case MG_ERR_DEVICE: return "device error";
    case MG_ERR_UNSUPPORTED: return "unsupported";
    case MG_ERR_BUSY: return "busy";
    case MG_ERR_CANCELLED: return "cancelled";
    default: return "unknown status";
  }
}

const char* mg_last_error(const mg_sim* sim) {
  return sim ? sim->err.c_str() : g_create_error.c_str();
}

mg_status mg_create(const mg_config* cfg, mg_sim** out) {
  if (!out) return fail(nullptr, MG_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg) return fail(nullptr, MG_ERR_INVALID, "cfg is NULL");
  if (cfg->abi_version != MG_ABI_VERSION) return fail(nullptr, MG_ERR_INVALID, "ABI version mismatch");
  // at most 2^30 - 1024 envs, so that a padded row of floats stays below 4 GiB
  // and the step kernel addresses it with 32-bit lane offsets (2^30 envs would
  // not fit in device memory anyway: about 296 bytes each)
  if (cfg->n_envs < 1 || cfg->n_envs > ((int64_t)1 << 30) - 1024)
    return fail(nullptr, MG_ERR_INVALID, "n_envs outside 1 .. 2^30 - 1024");
  if (cfg->n_classes < 1 || cfg->n_classes > MG_MAX_CLASSES || !cfg->classes)
    return fail(nullptr, MG_ERR_INVALID, "n_classes outside 1..16 or classes NULL");
  if (!(cfg->dt_sub > 0.0) || !std::isfinite(cfg->dt_sub) || cfg->substeps < 1)
    return fail(nullptr, MG_ERR_INVALID, "dt_sub must be > 0 and substeps >= 1");
  for (int k = 0; k < cfg->n_classes; ++k) {
    std::string why;
    bool unsup;
    mg_status st = validate_vehicle(cfg->classes[k], k, why, unsup);
    if (st) return fail(nullptr, st, why);
  }
  const int64_t E = cfg->n_envs;
  std::vector<int64_t> count(cfg->n_classes, 0);
  if (cfg->env_class) {
    for (int64_t e = 0; e < E; ++e) {
      const int32_t c = cfg->env_class[e];
      if (c < 0 || c >= cfg->n_classes) return fail(nullptr, MG_ERR_INVALID, "env_class out of range");
      ++count[c];
    }
  } else {
    count[0] = E;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(nullptr, MG_ERR_DEVICE, "no HIP device");
  }
  if (cfg->device < 0 || cfg->device >= ndev) return fail(nullptr, MG_ERR_INVALID, "bad device ordinal");

  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, cfg->device) != hipSuccess ||
      n_cu < 1) {
    (void)hipGetLastError();
    return fail(nullptr, MG_ERR_DEVICE, "cannot query the device's compute units");
  }

  mg_sim* s = new mg_sim();
  s->device = cfg->device;
  s->n_cu = n_cu;
  s->stream = (hipStream_t)cfg->stream;
  s->E = E;
  s->n_classes = cfg->n_classes;
  s->substeps = cfg->substeps;
  s->dt = cfg->dt_sub;
  int32_t dmax = 13, nmax = 1;
  for (int k = 0; k < cfg->n_classes; ++k) {
    const mg_vehicle& v = cfg->classes[k];
    s->cc.push_back(make_class_const(v, cfg->dt_sub, cfg->substeps));
    s->nominal.push_back(make_nominal(v));
    nmax = std::max(nmax, v.n_thr);
    if (v.thr_tau > 0.0) dmax = std::max(dmax, 13 + v.n_thr);
  }
  s->D = dmax;
  s->n_max = nmax;
  // class segments, each starting on a wavefront boundary
  int64_t off = 0;
  int32_t blk = 0;
  for (int k = 0; k < cfg->n_classes; ++k) {
    s->seg_start.push_back(off);
    s->seg_len.push_back(count[k]);
    s->seg_blk_off.push_back(blk);
    blk += (int32_t)((count[k] + kBlock - 1) / kBlock);
    off += (count[k] + kSegAlign - 1) / kSegAlign * kSegAlign;
  }
  s->Ep = std::max<int64_t>(off, kSegAlign);
  s->nblk_total = blk;
  std::vector<int32_t> perm(s->Ep, -1), iperm(E);
  std::vector<uint8_t> cls(s->Ep, 0);
  {
    std::vector<int64_t> fill(s->seg_start);
    for (int64_t e = 0; e < E; ++e) {
      const int32_t c = cfg->env_class ? cfg->env_class[e] : 0;
      const int64_t j = fill[c]++;
      perm[j] = (int32_t)e;
      iperm[e] = (int32_t)j;
    }
    for (int k = 0; k < cfg->n_classes; ++k)
      for (int64_t j = s->seg_start[k]; j < s->seg_start[k] + ((count[k] + kSegAlign - 1) / kSegAlign) * kSegAlign; ++j)
        cls[j] = (uint8_t)k;
  }
  bool identity = true;
  for (int64_t e = 0; e < E && identity; ++e) identity = iperm[e] == e;

  DeviceGuard g(s->device);
  auto bail = [&](mg_status code, const std::string& msg) {
    g_create_error = msg;
    mg_destroy(s);
    return code;
  };
  const size_t Ep = (size_t)s->Ep;
  if (hipMalloc(&s->state, Ep * s->D * sizeof(float)) != hipSuccess ||
      hipMalloc(&s->params, Ep * kNumParams * sizeof(float)) != hipSuccess ||
      hipMalloc(&s->derived, Ep * kNumDerived * sizeof(float)) != hipSuccess ||
      hipMalloc(&s->class_of, Ep) != hipSuccess || hipMalloc(&s->flags, Ep) != hipSuccess ||
      hipMalloc(&s->nominal_dev, sizeof(ClassNominal) * s->n_classes) != hipSuccess ||
      hipMalloc(&s->staging, (size_t)E * std::max(s->D, kNumParams) * sizeof(float)) != hipSuccess ||
      (!identity && (hipMalloc(&s->perm, Ep * sizeof(int32_t)) != hipSuccess ||
                     hipMalloc(&s->iperm, (size_t)E * sizeof(int32_t)) != hipSuccess))) {
    (void)hipGetLastError();
    return bail(MG_ERR_OOM, "device allocation failed in mg_create");
  }
  if (hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      hipMemset(s->state, 0, Ep * s->D * sizeof(float)) != hipSuccess ||
      hipMemset(s->params, 0, Ep * kNumParams * sizeof(float)) != hipSuccess ||
      hipMemset(s->derived, 0, Ep * kNumDerived * sizeof(float)) != hipSuccess ||
      hipMemset(s->flags, 0, Ep) != hipSuccess ||
      hipMemcpy(s->class_of, cls.data(), Ep, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(s->nominal_dev, s->nominal.data(), sizeof(ClassNominal) * s->n_classes,
                hipMemcpyHostToDevice) != hipSuccess ||
      (!identity && (hipMemcpy(s->perm, perm.data(), Ep * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
                     hipMemcpy(s->iperm, iperm.data(), (size_t)E * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess))) {
    (void)hipGetLastError();
    return bail(MG_ERR_DEVICE, "device initialisation failed in mg_create");
  }
  // the debug build's failed-check word; MG_DEBUG_SHRINK=k (read here, debug
  // build only) makes the kernels treat caller columns >= E - k as out of
  // bounds, so that a test can see the checks fire while every access stays in
  // bounds (those lanes only skip their work)
  s->dbg.cols = E;
  s->dbg.list = 0;
#ifdef MG_DEBUG
  if (hipMalloc(&s->dbg.word, sizeof(uint32_t)) != hipSuccess ||
      hipMemset(s->dbg.word, 0, sizeof(uint32_t)) != hipSuccess) {
    (void)hipGetLastError();
    return bail(MG_ERR_OOM, "debug word allocation failed in mg_create");
  }
  if (const char* sh = std::getenv("MG_DEBUG_SHRINK"))
    s->dbg.cols = std::max<int64_t>(0, E - std::atoll(sh));
#endif
  for (int k = 1; k < s->n_classes; ++k) {
    hipStream_t hs = nullptr;
    hipEvent_t e1 = nullptr, e2 = nullptr;
    if (hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&e2, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      if (hs) s->aux.push_back(hs);
      if (e1) s->ev_fork.push_back(e1);
      if (e2) s->ev_join.push_back(e2);
      return bail(MG_ERR_DEVICE, "helper stream creation failed in mg_create");
    }
    s->aux.push_back(hs);
    s->ev_fork.push_back(e1);
    s->ev_join.push_back(e2);
  }
  if (reset_impl(s, nullptr, E, nullptr, nullptr, 0, 1) != MG_OK ||
      hipStreamSynchronize(s->stream) != hipSuccess) {
    (void)hipGetLastError();
    return bail(MG_ERR_DEVICE, "initial reset failed: " + s->err);
  }
  // set-up of mg_adj_backward_noalloc: the device address of its static
  // scratch, looked up once per device while that device is current
  if (!noalloc_scratch(s->device))
    return bail(MG_ERR_DEVICE, "cannot look up the static adjoint scratch on this device");
  *out = s;
  return MG_OK;
}

void mg_destroy(mg_sim* s) {
  if (!s) return;
  {
    DeviceGuard g(s->device);
    if (s->stream || s->state) (void)hipStreamSynchronize(s->stream);
    clear_graphs(s);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    for (hipStream_t h : s->aux) (void)hipStreamDestroy(h);
    for (hipEvent_t e : s->ev_fork) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->ev_join) (void)hipEventDestroy(e);
    void* bufs[] = {s->state, s->params, s->derived, s->perm, s->iperm, s->class_of, s->flags,
                    s->nominal_dev, s->partials, s->staging, s->segbuf, s->task_f, s->task_k,
                    s->split_acc, s->dbg.word};
    for (void* b : bufs)
      if (b) (void)hipFree(b);
    (void)hipGetLastError();
  }
  delete s;
}

mg_status mg_set_stream(mg_sim* s, void* stream) {
  if (!s) return MG_ERR_INVALID;
  s->stream = (hipStream_t)stream;
  return MG_OK;
}

int32_t mg_state_dim(const mg_sim* s) { return s ? s->D : -1; }
int32_t mg_action_dim(const mg_sim* s) { return s ? s->n_max : -1; }
int64_t mg_num_envs(const mg_sim* s) { return s ? s->E : -1; }

mg_status mg_reset(mg_sim* s, const int64_t* env_ids, int64_t n_ids, const float* state,
                   const float* param_mult) {
  mg_status st = check_usable(s);
  if (st) return st;
  int64_t n = n_ids;
  if (!env_ids) {
    if (n_ids != 0 && n_ids != s->E) return fail(s, MG_ERR_INVALID, "n_ids must be 0 or n_envs when env_ids is NULL");
    n = s->E;
  } else if (n_ids < 0) {
    return fail(s, MG_ERR_INVALID, "n_ids < 0");
  }
  DeviceGuard g(s->device);
  return reset_impl(s, env_ids, n, state, param_mult, 0, 1);
}

mg_status mg_set_params(mg_sim* s, const float* params) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!params) return fail(s, MG_ERR_INVALID, "params is NULL");
  DeviceGuard g(s->device);
  return reset_impl(s, nullptr, s->E, nullptr, params, 1, 0);
}

mg_status mg_set_state(mg_sim* s, const float* state) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!state) return fail(s, MG_ERR_INVALID, "state is NULL");
  DeviceGuard g(s->device);
  if (!s->perm) {
    MG_HIP(s, hipMemcpy2DAsync(s->state, s->Ep * sizeof(float), state, s->E * sizeof(float),
                               s->E * sizeof(float), s->D, hipMemcpyDeviceToDevice, s->stream));
  } else {
    MG_HIP(s, launch_scatter_in(state, s->E, s->state, s->Ep, s->D, s->perm, s->Ep, s->stream));
  }
  // new states: no env is frozen for its state any more
  MG_HIP(s, launch_flags_mask(s->flags, s->Ep, (uint8_t)~kFlagNonFinite, s->stream));
  return MG_OK;
}

mg_status mg_get_flags(mg_sim* s, int32_t* out, int32_t out_on_device) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!out) return fail(s, MG_ERR_INVALID, "out is NULL");
  DeviceGuard g(s->device);
  int32_t* dst = out_on_device ? out : reinterpret_cast<int32_t*>(s->staging);
  MG_HIP(s, launch_flags_out(s->flags, dst, s->E, s->perm, s->Ep, s->stream));
  if (!out_on_device) {
    MG_HIP(s, hipMemcpyAsync(out, s->staging, (size_t)s->E * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s->stream));
    MG_HIP(s, hipStreamSynchronize(s->stream));
  }
  return MG_OK;
}

int32_t mg_debug_build(void) {
#ifdef MG_DEBUG
  return 1;
#else
  return 0;
#endif
}

mg_status mg_debug_word(mg_sim* s, uint32_t* word, int32_t clear) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!word) return fail(s, MG_ERR_INVALID, "word is NULL");
  *word = 0;
  if (!s->dbg.word) return MG_OK;
  DeviceGuard g(s->device);
  MG_HIP(s, hipStreamSynchronize(s->stream));
  MG_HIP(s, hipMemcpy(word, s->dbg.word, sizeof(uint32_t), hipMemcpyDeviceToHost));
  if (clear) MG_HIP(s, hipMemset(s->dbg.word, 0, sizeof(uint32_t)));
  return MG_OK;
}

mg_status mg_step(mg_sim* s, const float* actions, int32_t n_ctrl, const float* targets,
                  float* traj, double* stats) {
  return step_common(s, actions, n_ctrl, targets, traj, stats, false);
}

mg_status mg_step_split(mg_sim* s, const float* actions, int32_t n_ctrl, float* traj) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!actions) return fail(s, MG_ERR_INVALID, "actions is NULL");
  if (n_ctrl < 1) return fail(s, MG_ERR_INVALID, "n_ctrl must be >= 1");
  DeviceGuard g(s->device);
  if (!s->split_acc) {
    if (hipMalloc(&s->split_acc, (size_t)6 * s->Ep * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(s, MG_ERR_OOM, "split-scheme accelerations");
    }
    MG_HIP(s, hipMemsetAsync(s->split_acc, 0, (size_t)6 * s->Ep * sizeof(float), s->stream));
  }
  SplitArgs a;
  std::memset(&a, 0, sizeof(a));
  a.state = s->state;
  MG_SET_DBG(a, s->dbg);
  a.params = s->params;
  a.derived = s->derived;
  a.acc = s->split_acc;
  a.Ep = s->Ep;
  a.E = s->E;
  a.perm = s->perm;
  a.actions = actions;
  a.n_max = s->n_max;
  a.D = s->D;
  a.n_ctrl = n_ctrl;
  a.substeps = s->substeps;
  a.traj = traj;
  a.dt = (float)s->dt;
  hipStream_t st0 = s->stream;
  for (int k = 1; k < s->n_classes; ++k) {
    MG_HIP(s, hipEventRecord(s->ev_fork[k - 1], st0));
    MG_HIP(s, hipStreamWaitEvent(s->aux[k - 1], s->ev_fork[k - 1], 0));
  }
  for (int k = 0; k < s->n_classes; ++k) {
    a.seg_start = s->seg_start[k];
    a.seg_len = s->seg_len[k];
    a.zg = s->nominal[k].zg;
    MG_HIP(s, launch_split(s->cc[k], a, k == 0 ? st0 : s->aux[k - 1]));
  }
  for (int k = 1; k < s->n_classes; ++k) {
    MG_HIP(s, hipEventRecord(s->ev_join[k - 1], s->aux[k - 1]));
    MG_HIP(s, hipStreamWaitEvent(st0, s->ev_join[k - 1], 0));
  }
  return MG_OK;
}

mg_status mg_task_configure(mg_sim* s, const mg_task* task, const float* center,
                            const float* phase, const float* yaw) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!task || !center || !phase) return fail(s, MG_ERR_INVALID, "task, center and phase are required");
  if (task->task < MG_TASK_STATION || task->task > MG_TASK_LEMNISCATE)
    return fail(s, MG_ERR_INVALID, "unknown task");
  if (task->task != MG_TASK_STATION && (task->lookahead < 1 || task->lookahead > MG_MAX_LOOKAHEAD))
    return fail(s, MG_ERR_INVALID, "lookahead outside 1..MG_MAX_LOOKAHEAD");
  if (task->episode_steps < 1) return fail(s, MG_ERR_INVALID, "episode_steps must be >= 1");
  const double vals[] = {task->radius, task->omega, task->climb_rate, task->lookahead_dt,
                         task->max_error};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(s, MG_ERR_INVALID, "non-finite task parameter");
  if (task->max_error < 0.0) return fail(s, MG_ERR_INVALID, "max_error must be >= 0");
  DeviceGuard g(s->device);
  if (!s->task_f) {
    if (hipMalloc(&s->task_f, (size_t)5 * s->Ep * sizeof(float)) != hipSuccess ||
        hipMalloc(&s->task_k, (size_t)s->Ep * sizeof(int32_t)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(s, MG_ERR_OOM, "task buffers");
    }
    MG_HIP(s, hipMemsetAsync(s->task_f, 0, (size_t)5 * s->Ep * sizeof(float), s->stream));
  }
  if ((st = copy_in(s, center, 3, s->task_f))) return st;
  if ((st = copy_in(s, phase, 1, s->task_f + 3 * s->Ep))) return st;
  if (yaw) {
    if ((st = copy_in(s, yaw, 1, s->task_f + 4 * s->Ep))) return st;
  } else {
    MG_HIP(s, hipMemsetAsync(s->task_f + 4 * s->Ep, 0, (size_t)s->Ep * sizeof(float), s->stream));
  }
  MG_HIP(s, hipMemsetAsync(s->task_k, 0, (size_t)s->Ep * sizeof(int32_t), s->stream));
  TaskConst& tc = s->task;
  tc.task = task->task;
  tc.m = task->task == MG_TASK_STATION ? 1 : task->lookahead;
  tc.L = task->episode_steps;
  tc.R = task->radius;
  tc.omega = task->omega;
  tc.climb = task->climb_rate;
  tc.dtc = s->dt * s->substeps;
  tc.dl = task->lookahead_dt > 0.0 ? task->lookahead_dt : tc.dtc;
  tc.emax = task->max_error;
  tc.cdl = std::cos(tc.omega * tc.dl);
  tc.sdl = std::sin(tc.omega * tc.dl);
  s->task_on = true;
  return MG_OK;
}

int32_t mg_task_obs_dim(const mg_sim* s) {
  if (!s || !s->task_on) return 0;
  return s->task.task == MG_TASK_STATION ? 12 : 6 * s->task.m + 6;
}

mg_status mg_task_observe(mg_sim* s, float* obs) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!s->task_on) return fail(s, MG_ERR_INVALID, "no task configured");
  if (!obs) return fail(s, MG_ERR_INVALID, "obs is NULL");
  DeviceGuard g(s->device);
  return enqueue_task(s, nullptr, obs, nullptr, nullptr, nullptr, nullptr);
}

mg_status mg_task_step(mg_sim* s, const float* actions, float* obs, float* err, int32_t* done,
                       const float* reset_state, const float* reset_mult) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!s->task_on) return fail(s, MG_ERR_INVALID, "no task configured");
  if (!actions || !obs) return fail(s, MG_ERR_INVALID, "actions and obs are required");
  DeviceGuard g(s->device);
  return enqueue_task(s, actions, obs, err, done, reset_state, reset_mult);
}

mg_status mg_task_counters(mg_sim* s, int32_t* out) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!s->task_on) return fail(s, MG_ERR_INVALID, "no task configured");
  DeviceGuard g(s->device);
  // the layout copy moves 32-bit words unchanged, so it serves int32 rows too
  return copy_out(s, reinterpret_cast<const float*>(s->task_k), 1, reinterpret_cast<float*>(out), 1);
}

mg_status mg_step_plain(mg_sim* s, const float* actions, int32_t n_ctrl, const float* targets,
                        float* traj, double* stats) {
  return step_common(s, actions, n_ctrl, targets, traj, stats, true);
}

mg_status mg_rollout(mg_sim* s, const float* actions, int32_t T, const float* targets,
                     float* traj, double* stats, int32_t plain) {
  mg_status st = check_usable(s);
  if (st) return st;
  if (!actions) return fail(s, MG_ERR_INVALID, "actions is NULL");
  if (T < 1) return fail(s, MG_ERR_INVALID, "T must be >= 1");
  DeviceGuard g(s->device);
  if (stats && (st = ensure_partials(s, T))) return st;
  GraphKey key{T, plain ? 1 : 0, actions, targets, traj, stats};
  auto it = s->graphs.find(key);
  if (it == s->graphs.end()) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    MG_HIP(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    mg_status est = enqueue_steps(s, s->cap_stream, actions, T, targets, traj, stats, plain != 0, true);
    hipError_t ce = hipStreamEndCapture(s->cap_stream, &graph);
    if (est) {
      if (graph) (void)hipGraphDestroy(graph);
      return est;
    }
    if (ce != hipSuccess) return fail(s, MG_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(s, MG_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
    if (s->graphs.size() >= kMaxCachedGraphs) {
      // bounded cache: a caller cycling through many buffers starts it afresh
      MG_HIP(s, hipStreamSynchronize(s->stream));
      clear_graphs(s);
    }
    it = s->graphs.emplace(key, exec).first;
  }
  MG_HIP(s, hipGraphLaunch(it->second, s->stream));
  return MG_OK;
}

mg_status mg_get_state(mg_sim* s, float* out, int32_t out_on_device) {
  mg_status st = check_usable(s);
  if (st) return st;
  DeviceGuard g(s->device);
  return copy_out(s, s->state, s->D, out, out_on_device);
}

mg_status mg_get_params(mg_sim* s, float* out, int32_t out_on_device) {
  mg_status st = check_usable(s);
  if (st) return st;
  DeviceGuard g(s->device);
  return copy_out(s, s->params, kNumParams, out, out_on_device);
}

mg_status mg_adj_forward(mg_sim* s, const float* actions, int32_t T, int32_t ckpt_every,
                         float* ckpt, float* traj) {
  mg_status st = adj_common(s, actions, T, ckpt_every, ckpt);
  if (st) return st;
  DeviceGuard g(s->device);
  AdjArgs a = adj_args(s, actions, T, ckpt_every);
  a.ckpt = ckpt;
  a.traj = traj;
  for (int k = 0; k < s->n_classes; ++k) {
    a.seg_start = s->seg_start[k];
    a.seg_len = s->seg_len[k];
    MG_HIP(s, launch_adjoint(false, s->cc[k], a, s->stream));
  }
  return MG_OK;
}

mg_status mg_adj_backward(mg_sim* s, const float* ckpt, const float* traj, const float* actions,
                          int32_t T, int32_t ckpt_every, const float* dL_dtraj, float* dL_dact,
                          float* dL_dtheta, float* dL_dx0) {
  mg_status st = adj_common(s, actions, T, ckpt_every, ckpt);
  if (st) return st;
  if (!dL_dtraj || !dL_dact || !dL_dtheta)
    return fail(s, MG_ERR_INVALID, "dL_dtraj, dL_dact and dL_dtheta must not be NULL");
  DeviceGuard g(s->device);
  // with one sub-step per control step, the forward's trajectory holds every
  // sub-step input: for launches of at most one wave per SIMD nothing is then
  // recomputed and no scratch is used
  if (traj_inputs(s, traj))
    return adj_backward_launch(s, ckpt, traj, actions, T, ckpt_every, dL_dtraj, dL_dact,
                               dL_dtheta, dL_dx0, nullptr, true);
  // When the rollout's sub-step inputs fit in 4 GiB, every segment is
  // recomputed at once into a whole-rollout buffer and the backward only
  // sweeps: a sparse launch then waits for one segment's recomputation
  // instead of each in turn (8192 envs, 64 control steps: backward 0.32 ->
  // 0.26 ms), and a crowded one runs a sweep kernel without the
  // recomputation's registers (2^20 envs: 5.1 -> 4.8 ms).  Otherwise each
  // segment is recomputed just before its sweep into a segment-sized buffer;
  // so is every segment when the whole-rollout buffer cannot be allocated.
  const int32_t nseg = (T + ckpt_every - 1) / ckpt_every;
  const size_t whole_floats = (size_t)T * s->substeps * s->D * (size_t)s->Ep;
  const size_t seg_floats = (size_t)std::min(ckpt_every, T) * s->substeps * s->D * (size_t)s->Ep;
  bool whole = nseg > 1 && nseg <= 65535 && whole_floats * sizeof(float) <= ((size_t)4 << 30);
  if (whole && whole_floats > s->segbuf_cap) {
    // the new buffer is allocated before the old one is released, so that a
    // failure leaves the old one in place
    MG_HIP(s, hipStreamSynchronize(s->stream));
    float* nb = nullptr;
    if (hipMalloc(&nb, whole_floats * sizeof(float)) == hipSuccess) {
      float* old = s->segbuf;
      s->segbuf = nb;
      s->segbuf_cap = whole_floats;
      if (old) MG_HIP(s, hipFree(old));
    } else {
      (void)hipGetLastError();
      whole = false;
    }
  }
  if (!whole && seg_floats > s->segbuf_cap) {
    MG_HIP(s, hipStreamSynchronize(s->stream));
    if (s->segbuf) MG_HIP(s, hipFree(s->segbuf));
    s->segbuf = nullptr;
    s->segbuf_cap = 0;
    if (hipMalloc(&s->segbuf, seg_floats * sizeof(float)) != hipSuccess) {
      (void)hipGetLastError();
      s->segbuf = nullptr;
      return fail(s, MG_ERR_OOM, "adjoint scratch allocation failed");
    }
    s->segbuf_cap = seg_floats;
  }
  return adj_backward_launch(s, ckpt, nullptr, actions, T, ckpt_every, dL_dtraj, dL_dact,
                             dL_dtheta, dL_dx0, s->segbuf, whole);
}

mg_status mg_adj_backward_noalloc(mg_sim* s, const float* ckpt, const float* traj,
                                  const float* actions, int32_t T, int32_t ckpt_every,
                                  const float* dL_dtraj, float* dL_dact, float* dL_dtheta,
                                  float* dL_dx0) {
  mg_status st = adj_common(s, actions, T, ckpt_every, ckpt);
  if (st) return st;
  if (!dL_dtraj || !dL_dact || !dL_dtheta)
    return fail(s, MG_ERR_INVALID, "dL_dtraj, dL_dact and dL_dtheta must not be NULL");
  if (traj_inputs(s, traj)) {
    DeviceGuard g(s->device);
    return adj_backward_launch(s, ckpt, traj, actions, T, ckpt_every, dL_dtraj, dL_dact,
                               dL_dtheta, dL_dx0, nullptr, true);
  }
  // the same choice as mg_adj_backward, bounded by the static scratch instead
  // of by what can be allocated
  const size_t cap = MG_NOALLOC_SCRATCH_BYTES / sizeof(float);
  const int32_t nseg = (T + ckpt_every - 1) / ckpt_every;
  const size_t whole_floats = (size_t)T * s->substeps * s->D * (size_t)s->Ep;
  const size_t seg_floats = (size_t)std::min(ckpt_every, T) * s->substeps * s->D * (size_t)s->Ep;
  const bool whole = nseg > 1 && nseg <= 65535 && whole_floats <= cap;
  if (!whole && seg_floats > cap)
    return fail(s, MG_ERR_INVALID,
                "mg_adj_backward_noalloc: one segment's sub-step states (" +
                    std::to_string(seg_floats * sizeof(float)) + " bytes) exceed the " +
                    std::to_string((size_t)MG_NOALLOC_SCRATCH_BYTES) +
                    "-byte static scratch; use a smaller ckpt_every or mg_adj_backward");
  DeviceGuard g(s->device);
  float* buf = g_noalloc_ptr[s->device];   // set by mg_create on this device
  if (!buf) return fail(s, MG_ERR_DEVICE, "static adjoint scratch not set up on this device");
  return adj_backward_launch(s, ckpt, nullptr, actions, T, ckpt_every, dL_dtraj, dL_dact,
                             dL_dtheta, dL_dx0, buf, whole);
}

mg_status mg_synchronize(mg_sim* s) {
  mg_status st = check_usable(s);
  if (st) return st;
  DeviceGuard g(s->device);
  MG_HIP(s, hipStreamSynchronize(s->stream));
  MG_HIP(s, hipGetLastError());
  return MG_OK;
}

}  // extern "C"
