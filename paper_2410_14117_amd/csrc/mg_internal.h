// mg_internal.h -- structures shared by the host runtime and the kernel
// translation units of libmg (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "mg.h"

namespace mg {

constexpr int kMaxThr = 8;
constexpr int kNumParams = 23;
constexpr int kNumDerived = 30;
constexpr int kNumTheta = 19;
#ifndef MG_BLOCK
#define MG_BLOCK 256
#endif
constexpr int kBlock = MG_BLOCK; // threads per block of the step kernels (4 wave64)
constexpr int kSegAlign = 64;    // each class segment starts on a wavefront boundary
constexpr double kG0 = 9.81;

// Rows of the per-env derived-constant table [kNumDerived][Ep], formed once at
// reset.  With I_g and M_A diagonal and r_g = (0,0,z_g) the mass matrix only
// couples (u,q) and (v,p), so M and M^-1 have 8 distinct entries each.
enum DerivedRow : int {
  kMuu = 0, kMvv, kMww, kMpp, kMqq, kMrr, kMuq, kMvp,     // M
  kIuu = 8, kIvv, kIww, kIpp, kIqq, kIrr, kIuq, kIvp,     // M^-1
  kDL = 16,                                               // 6 rows
  kDQ = 22,                                               // 6 rows
  kWmB = 28,                                              // W - B
  kHz = 29,                                               // W z_g - B z_b
};

// Wave-uniform constants of one vehicle class, passed by value (kernarg ->
// scalar registers).
struct ClassConst {
  float B[6][kMaxThr];   // allocation matrix
  float f_max;
  float inv_tau;         // 1 / thruster lag (0 if none)
  // Classical RK4 applied to the linear lag f' = (f_cmd - f) / tau with the
  // command held: with z = dt / tau the stage values are
  //   f_cmd + sigma_i (f - f_cmd),  sigma = 1, 1 - z/2, 1 - z/2 + z^2/4, 1 - z + z^2/2 - z^3/4
  // and one sub-step maps f - f_cmd to rho (f - f_cmd), rho = 1 - z + z^2/2 - z^3/6 + z^4/24.
  float sigma2, sigma3, sigma4, rho;
  int32_t n_thr;
  int32_t thr_map;       // 0 linear, 1 quadratic
  int32_t lag;
  float rho_s;           // rho^S for the owner's S sub-steps per control step
};

// Class constants for sub-steps of dt, S sub-steps per control step.  The
// allocation matrix is formed from the thruster geometry: column i is
// [d_i ; r_i x d_i].
ClassConst make_class_const(const mg_vehicle& v, double dt, int substeps);

// Nominal parameters of a class for the reset kernel (device table).
struct ClassNominal {
  double p[kNumParams];
  double zg, zb;
  int32_t n_thr, lag;
};

// per-env status flags (internal [Ep] bytes): the state went non-finite in a
// step (the env is then frozen), the mass matrix is not positive definite
constexpr uint8_t kFlagNonFinite = 1;
constexpr uint8_t kFlagNotSPD = 2;

// Debug build (compiled with -DMG_DEBUG, libmg_debug.so): the kernels check
// the indices their lanes address against the bounds of the buffers, and a
// failed check sets its bit in the device word `word` and the lane does no
// work, so a failed check never leads to an access out of bounds.  In the
// release build dbg_check is `true` and the checks compile to nothing.
constexpr uint32_t kDbgSegment = 1;  // a class segment reaches past the padded stride Ep
constexpr uint32_t kDbgColumn = 2;   // a caller column (perm, reset ids) outside [0, cols)
constexpr uint32_t kDbgInternal = 4; // an internal column (iperm) outside [0, Ep)
constexpr uint32_t kDbgList = 8;     // a tick-list entry outside the list
constexpr uint32_t kDbgPage = 16;    // a page column outside its request's arrays
struct DebugArgs {
  uint32_t* word;  // device word of failed-check bits (debug build), else NULL
  int64_t cols;    // bound of caller columns: E (lower under MG_DEBUG_SHRINK, a test hook)
  int64_t list;    // entries of the serving tick list
};
__device__ __forceinline__ bool dbg_check(const DebugArgs& d, bool ok, uint32_t bit) {
  if (!ok) atomicOr(d.word, bit);
  return ok;
}
// The argument structs carry `dbg` in the debug build only, so that the
// release build's kernels are the same code as without the checks; MG_CHECK
// (args, condition, bit) is `true` there and its operands are not evaluated.
// MG_CHECK_WITH(d, condition, bit) does the same with a DebugArgs d.
#ifdef MG_DEBUG
#define MG_DBG_FIELD DebugArgs dbg;
#define MG_CHECK_WITH(d, ok, bit) ::mg::dbg_check((d), (ok), (bit))
#define MG_CHECK(args, ok, bit) ::mg::dbg_check((args).dbg, (ok), (bit))
#define MG_SET_DBG(args, value) ((args).dbg = (value))
#else
#define MG_DBG_FIELD
#define MG_CHECK_WITH(d, ok, bit) true
#define MG_CHECK(args, ok, bit) true
#define MG_SET_DBG(args, value) ((void)0)
#endif

struct StepArgs {
  float* state;                // internal [D][Ep]
  uint8_t* flags;              // internal [Ep] status flags (read, set when an env freezes)
  const float* derived;        // internal [kNumDerived][Ep]
  int64_t Ep;                  // internal row stride
  int64_t E;                   // caller row stride
  const int32_t* perm;         // internal -> caller index, NULL = identity
  int64_t seg_start, seg_len;  // this class's internal range
  const float* actions;        // caller [n_ctrl][n_max][E]
  int32_t n_max;
  const float* targets;        // caller [3][E] or NULL
  float* traj;                 // caller [n_ctrl][D][E] or NULL
  int32_t D;                   // I/O state width
  double* partials;            // [n_ctrl][nblk_total][4] or NULL
  int32_t nblk_total, blk_off;
  int32_t n_ctrl, substeps;
  float dt;
  MG_DBG_FIELD
};

struct ResetArgs {
  float* state;                // internal [D][Ep]
  uint8_t* flags;              // internal [Ep]: kFlagNotSPD from the new parameters; the
                               // non-finite flag cleared where the state is written
  float* params;               // internal [23][Ep] absolute
  float* derived;              // internal [kNumDerived][Ep]
  int64_t Ep, E;
  int32_t D;
  const int32_t* iperm;        // caller -> internal, NULL = identity
  const uint8_t* class_of;     // internal [Ep] class of each env
  const ClassNominal* nominal; // device [n_classes]
  const int64_t* ids;          // caller ids [n] or NULL (= 0..n-1)
  int64_t n;
  const float* state_in;       // [D][n] or NULL (rest)
  const float* param_in;       // [23][n] or NULL (nominal)
  int32_t param_absolute;      // param_in holds absolute values (else multipliers)
  int32_t write_state;         // 0: keep the state
  int32_t* task_k;             // internal [Ep] episode counters zeroed with the state, or NULL
  float* split_acc;            // internal [6][Ep] split-scheme accelerations zeroed likewise, or NULL
  MG_DBG_FIELD
};

// Gym-style task of Sec. III (wave-uniform, by value): kind, look-ahead
// count m, episode length L, curve radius, parameter rate, helix vertical
// rate, look-ahead spacing and control-step duration (s), error bound (m),
// and cos / sin of the curve-parameter step omega dl between look-ahead points.
struct TaskConst {
  int32_t task, m, L, pad_;
  double R, omega, climb, dl, dtc, emax, cdl, sdl;
};

struct TaskArgs {
  float* state;                // internal [D][Ep]
  uint8_t* flags;              // internal [Ep]: cleared (kFlagNotSPD re-derived) on restart
  float* params;               // internal [23][Ep]
  float* derived;              // internal [kNumDerived][Ep]
  const float* task_f;         // internal [5][Ep]: centre x, y, z, curve phase, target yaw
  int32_t* task_k;             // internal [Ep] control steps since the episode began
  int64_t Ep, E;
  const int32_t* perm;         // internal -> caller, NULL = identity
  int64_t seg_start, seg_len;
  const ClassNominal* nominal; // device, this class's entry
  const float* actions;        // caller [n_max][E], or NULL: observe only
  int32_t n_max, D, substeps;
  float dt;
  float* obs;                  // caller [obs_dim][E]
  float* err;                  // caller [E] or NULL
  int32_t* done;               // caller [E] or NULL
  const float* reset_state;    // caller [D][E] or NULL (rest at the origin)
  const float* reset_mult;     // caller [23][E] or NULL (parameters kept)
  MG_DBG_FIELD
};

// The split scheme of Sec. II (rigid body by semi-implicit Euler, the
// hydrodynamic wrench with the previous sub-step's added-mass acceleration as
// an external force).
struct SplitArgs {
  float* state;                // internal [D][Ep]
  const float* params;         // internal [23][Ep] absolute
  const float* derived;        // internal [kNumDerived][Ep]
  float* acc;                  // internal [6][Ep] previous sub-step's acceleration
  int64_t Ep, E;
  const int32_t* perm;
  int64_t seg_start, seg_len;
  const float* actions;        // caller [n_ctrl][n_max][E]
  int32_t n_max, D, n_ctrl, substeps;
  float* traj;                 // caller [n_ctrl][D][E] or NULL
  float dt;
  double zg;                   // this class's CG height below the CO
  MG_DBG_FIELD
};

struct AdjArgs {
  float* state;                // internal [D][Ep] (forward reads and advances it)
  const float* derived;        // internal [kNumDerived][Ep]
  int64_t Ep, E;
  const int32_t* perm;
  int64_t seg_start, seg_len;
  const float* actions;        // caller [T][n_max][E]
  int32_t n_max, D, T, substeps, ckpt_every;
  float dt;
  float* ckpt;                 // caller [ceil(T/K)][D][E]
  float* traj;                 // caller [T][D][E] or NULL: written by the forward; read by
                               // the backward when recomputed == 2
  const float* gtraj;          // caller [T][D][E] dL/d traj (backward)
  float* gact;                 // caller [T][n_max][E]
  float* gtheta;               // caller [19][E]
  float* gx0;                  // caller [D][E] or NULL
  float* segbuf;               // internal [K * S][Dc][Ep] scratch (Dc = class state width),
                               // or [T * S][Dc][Ep] when recomputed
  float zb;                    // class z_b (for dL/dB through h_z)
  int32_t n_cu;                // compute units (picks the backward kernel's occupancy)
  int32_t recomputed;          // 1: segbuf already holds every sub-step input of the rollout;
                               // 2: one sub-step per control step, inputs read from traj
  MG_DBG_FIELD
};

// ---- serving loop (kernels_serve.hip) -------------------------------------
// A page is a block of (Dmax + kNumDerived) rows x 64 lanes of floats: the
// state rows first, then the per-env derived constants; its column map gives,
// per lane, the env's column in the request's input arrays (-1 = empty lane).
// The per-tick item arrays (joins, leaves) live in pinned host memory that
// the kernels read through its device mapping: a tick copies nothing to the
// device.
struct ServeTickItem {         // one active page (device-resident list entry)
  float* block;                // NULL: an empty entry
  const int32_t* cols;
  const float* actions;        // request [L][n_max][ld], or NULL: generated from seed
  int64_t ld;
  int64_t t0;                  // control-step clock when the request joined
  int32_t L;                   // control steps of the request
  int32_t pad_;
  uint64_t seed;               // SplitMix64 seed of generated throttles
  int64_t n;                   // env count of the request (generated throttles)
};
struct ServeInitItem {         // one newly admitted page
  float* block;
  const int32_t* cols_src;     // staged column map of the page (64 entries)
  int32_t* cols;               // the page's own column map (written here)
  const float* x0;             // request [D][ld]
  const float* mult;           // request [23][ld] or NULL
  int64_t ld;
  int32_t cls;
  int32_t pad_;
  int64_t list_index;          // its tick-list entry, cls * capacity + entry,
  ServeTickItem item;          // which receives this item
};
struct ServeGatherItem {       // one page of a finished request
  const float* block;
  const int32_t* cols;
  float* out;                  // device staging [Dmax][n] of the request
  int64_t n;
  int64_t list_index;          // its tick-list entry, emptied here
};
struct ServeTickArgs {         // one tick over the pages of every class
  const ServeTickItem* list;   // [n_classes][list_cap]
  const ClassConst* cc;        // device [n_classes]
  int64_t list_cap;
  int64_t tick;                // control-step clock at the tick's start
  int32_t count[16];           // list entries in use per class
  int32_t n_classes;
  int32_t steps;               // most control steps a page advances
  int32_t Dmax, n_max, substeps;
  float dt;
  MG_DBG_FIELD
};
// joins: initialise each admitted page (one 64-lane block per page) and enter
// it in the tick list
hipError_t launch_serve_join(const ServeInitItem* items, int32_t n_items, ServeTickItem* list,
                             const ClassNominal* nominal, int32_t Dmax, const DebugArgs& dbg,
                             hipStream_t s);
// one launch advances the pages of all classes (a wave per page, persistent
// over `grid` blocks)
hipError_t launch_serve_tick(const ServeTickArgs& a, int32_t grid, hipStream_t s);
// leaves: copy each finished page's states into its request's staging and
// empty its tick-list entry
hipError_t launch_serve_leave(const ServeGatherItem* items, int32_t n_items, ServeTickItem* list,
                              int32_t Dmax, const DebugArgs& dbg, hipStream_t s);

// launchers (kernels_adjoint.hip)
hipError_t launch_adjoint(bool backward, const ClassConst& cc, const AdjArgs& a, hipStream_t s);
// every segment's sub-step inputs at once, into the whole-rollout segbuf
hipError_t launch_adj_recompute(const ClassConst& cc, const AdjArgs& a, hipStream_t s);

// launchers (kernels_step.hip)
hipError_t launch_step(const ClassConst& cc, const StepArgs& a, hipStream_t s);
hipError_t launch_stats_finalize(const double* partials, int32_t nblk, int32_t n_ctrl,
                                 double* stats, hipStream_t s);
hipError_t launch_reset(const ResetArgs& a, hipStream_t s);
hipError_t launch_task(const ClassConst& cc, const TaskConst& tc, const TaskArgs& a, hipStream_t s);
hipError_t launch_split(const ClassConst& cc, const SplitArgs& a, hipStream_t s);
// out[r][perm[j]] = in[r][j] for rows r < rows (internal -> caller order)
// status flags to caller order int32 [E]; flags &= mask for n envs
hipError_t launch_flags_out(const uint8_t* flags, int32_t* out, int64_t E, const int32_t* perm,
                            int64_t n_internal, hipStream_t s);
hipError_t launch_flags_mask(uint8_t* flags, int64_t n, uint8_t mask, hipStream_t s);
hipError_t launch_gather_out(const float* in, int64_t Ep, float* out, int64_t E, int32_t rows,
                             const int32_t* perm, int64_t n_internal, hipStream_t s);
// out[r][j] = in[r][perm[j]] (caller -> internal order), padding lanes untouched
hipError_t launch_scatter_in(const float* in, int64_t E, float* out, int64_t Ep, int32_t rows,
                             const int32_t* perm, int64_t n_internal, hipStream_t s);

}  // namespace mg
