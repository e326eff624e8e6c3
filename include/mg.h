/*
 * mg.h -- C ABI of the MI355X batched Fossen 6-DOF simulator (libmg.so).
 *
 * The library steps many independent underwater-vehicle environments through
 * Fossen's equation of motion as MarineGym states it (Sec. II "Method",
 * Eq. (1)): rigid-body plus added mass, rigid-body plus added-mass Coriolis,
 * linear plus quadratic damping, weight and buoyancy, driven by per-thruster
 * throttles (Eq. (3)) through a thruster allocation matrix, with several
 * sub-steps per control step (Sec. II, the paragraph after Eq. (1)), many
 * parallel environment instances and per-env domain randomisation (Sec. II,
 * first paragraph; Sec. III).  Integration is classical RK4 in FP32 with the
 * attitude quaternion renormalised after every sub-step.
 *
 * Conventions common to every call
 *   Units      SI.  World frame north-east-down, body frame forward-right-down,
 *              origin (CO) at the centre of buoyancy.
 *   State      one column per env, component-major (SoA) FP32:
 *                [x y z | qw qx qy qz | u v w p q r | f_1 .. f_n]
 *              p = NED position, q = Hamilton scalar-first unit quaternion
 *              body->NED, nu = body velocities, f = thruster states (present
 *              only for classes with a thruster lag).  The I/O width D =
 *              mg_state_dim() = 13 + the largest thruster count among lagged
 *              classes; rows a class does not use read as 0.
 *   Layout     every array argument is row-major [rows][n_envs] (or
 *              [frames][rows][n_envs]) in the caller's env order, FP32 unless
 *              stated; "device" pointers are HIP device memory of the sim's
 *              device, "host" pointers are ordinary host memory.
 *   Ownership  the sim owns every buffer it allocates; the caller owns every
 *              pointer it passes and keeps it alive until the work queued on
 *              the sim's stream has completed.
 *   Ordering   calls are enqueued on the sim's stream and return at once
 *              (except where "synchronous" is stated).
 *   Errors     every call returns an mg_status.  Argument errors return
 *              MG_ERR_INVALID with no side effect.  A failed HIP call makes
 *              the sim sticky: it and every later call return MG_ERR_DEVICE.
 *              An env whose state becomes non-finite is not an error: it is
 *              frozen and flagged (mg_get_flags) and counted in the episode
 *              statistics, and the rest of the batch steps on.
 *              mg_last_error() gives a text for the last failure.
 *   Threads    a sim is thread-compatible (one thread at a time); distinct
 *              sims may be used from distinct threads.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MG_ABI_VERSION 4u
#define MG_MAX_THRUSTERS 8
#define MG_MAX_CLASSES 16
#define MG_NUM_PARAMS 23  /* m, Ixx, Iyy, Izz, M_A(6), D_L(6), D_Q(6), B */
#define MG_NUM_THETA 19   /* differentiable subset: M_A(6), D_L(6), D_Q(6), B */
#define MG_NUM_STATS 4    /* sum dist, max dist, sum kinetic energy, non-finite count */

typedef int32_t mg_status;
#define MG_OK 0
#define MG_ERR_INVALID 1     /* bad argument; nothing was done */
#define MG_ERR_OOM 2         /* device allocation failed */
#define MG_ERR_DEVICE 3      /* a HIP call failed; the sim is unusable */
#define MG_ERR_UNSUPPORTED 4 /* valid description this GPU path does not implement */
#define MG_ERR_BUSY 5        /* server queue full / request not finished */
#define MG_ERR_CANCELLED 6   /* server request cancelled by mg_server_cancel */

typedef struct mg_sim mg_sim;

/* One vehicle class (Sec. II: BlueROV2 / BlueROV2 Heavy), raw preset numbers.
 *   mass, inertia  rigid-body mass (kg) and principal inertia about the CG (kg m^2)
 *   r_g, r_b       CG and CB w.r.t. the CO (m); the GPU path requires the x
 *                  and y components to be 0 (MG_ERR_UNSUPPORTED otherwise)
 *   added_mass     diagonal of M_A; d_lin, d_quad: diagonal linear and
 *                  quadratic damping; buoyancy B (N).  Weight W = 9.81 m.
 *   thr_pos/dir    position (m) and unit direction of positive thrust of each
 *                  of the n_thr (1..8) thrusters; column i of the allocation
 *                  matrix is [dir_i ; pos_i x dir_i]
 *   f_max          thrust at throttle 1 (N); thr_map 0: f = f_max a,
 *                  1: f = f_max a|a|, with a clamped to [-1, 1]
 *   thr_tau        first-order thruster lag (s); 0 = thrust follows the
 *                  command instantly (no thruster state) */
typedef struct {
  double mass, inertia[3], r_g[3], r_b[3], added_mass[6], d_lin[6], d_quad[6], buoyancy;
  double thr_pos[MG_MAX_THRUSTERS][3], thr_dir[MG_MAX_THRUSTERS][3], f_max, thr_tau;
  int32_t n_thr, thr_map;
} mg_vehicle;

/* Simulator description.
 *   abi_version  must be MG_ABI_VERSION
 *   n_envs       number of environments E (1 .. 2^30 - 1024)
 *   classes      host array of n_classes (1..MG_MAX_CLASSES) vehicles
 *   env_class    host [n_envs] class index per env, or NULL (all class 0);
 *                envs are regrouped internally so that every wavefront holds
 *                one class; the ABI always speaks the caller's env order
 *   dt_sub       RK4 sub-step (s) and substeps = sub-steps per control step
 *   device       HIP device ordinal; stream: hipStream_t or NULL (default) */
typedef struct {
  uint32_t abi_version;
  int32_t n_classes;
  int64_t n_envs;
  const mg_vehicle* classes;
  const int32_t* env_class;
  double dt_sub;
  int32_t substeps;
  int32_t device;
  void* stream;
} mg_config;

/* Library plumbing (no passage of the paper defines these): the ABI version
 * this library implements (MG_ABI_VERSION of its build), and a static text
 * for a status code ("unknown status" for codes it does not know). */
uint32_t mg_abi_version(void);
const char* mg_status_str(mg_status s);
/* Text of the last failure of this sim, or of the last failed mg_create when
 * sim is NULL.  Valid until the next call on the same sim. */
const char* mg_last_error(const mg_sim* sim);

/* The parallel environment instances of Sec. I (second contribution) and
 * Sec. II (component 1: BlueROV2 / BlueROV2 Heavy dynamics): allocates the
 * device buffers (state, parameters, derived constants) and leaves every env
 * at rest at the origin with nominal parameters (as mg_reset with NULL state
 * and multipliers).  Synchronous.  MG_ERR_INVALID for a malformed config,
 * MG_ERR_UNSUPPORTED for a class the GPU path does not implement, MG_ERR_OOM
 * if the buffers cannot be had; *out is NULL on any error. */
mg_status mg_create(const mg_config* cfg, mg_sim** out);
/* Ends the environment instances mg_create made (Sec. II, component 1):
 * waits for the sim's stream and frees everything the sim owns, never the
 * caller's buffers; NULL is ignored. */
void mg_destroy(mg_sim* sim);
/* The hipStream_t (or NULL: the default stream) every later call of this sim
 * is enqueued on, so that stepping orders itself with the learner's work on
 * the same GPU (Sec. III); NULL sim: MG_ERR_INVALID. */
mg_status mg_set_stream(mg_sim* sim, void* stream);
int32_t mg_state_dim(const mg_sim* sim);      /* D, or -1 for NULL */
int32_t mg_action_dim(const mg_sim* sim);     /* N_max = largest n_thr (Sec. II thrusters), or -1 */
int64_t mg_num_envs(const mg_sim* sim);       /* E, or -1 */

/* Domain randomisation and reset (Sec. II: physical-parameter randomisation).
 *   env_ids     device int64 [n_ids] caller env indices, or NULL for all envs
 *               (then n_ids must be 0 or E); out-of-range ids are skipped
 *   state       device [D][n_ids] new states, or NULL: at rest at the origin,
 *               identity attitude, zero thruster state
 *   param_mult  device [23][n_ids] multipliers of the class's nominal
 *               parameters, or NULL (nominal).  Here the per-env mass matrix
 *               M = M_RB + M_A and its inverse are formed once (in FP64,
 *               rounded to FP32) and kept for every later step; an env whose
 *               M is not positive definite (or whose parameters are not
 *               finite) gets NaN constants and the flag MG_FLAG_NOT_SPD, and
 *               is frozen until a reset gives it valid parameters.  The
 *               non-finite flag of every env whose state is written is
 *               cleared.  The check runs on the device, so mg_reset stays
 *               asynchronous and does not return MG_ERR_INVALID for it: read
 *               the flags to find such envs. */
mg_status mg_reset(mg_sim* sim, const int64_t* env_ids, int64_t n_ids, const float* state,
                   const float* param_mult);
/* Physical-parameter domain randomisation given as absolute values (Sec. II,
 * component 1): device [23][E] (same order as the multipliers), refactoring
 * M = M_RB + M_A of Eq. (1) as mg_reset does.  State is untouched.  Errors as
 * mg_reset (NULL params: MG_ERR_INVALID). */
mg_status mg_set_params(mg_sim* sim, const float* params);
/* Sets the pose eta and body velocity nu of Eq. (1) (Sec. II; as the
 * quaternion state described above) and the thruster states of every env
 * from device [D][E]; parameters are kept, MG_FLAG_NONFINITE is cleared.
 * Together with mg_get_state this is a bitwise-exact save and resume.  NULL
 * state: MG_ERR_INVALID. */
mg_status mg_set_state(mg_sim* sim, const float* state);

/* Per-env status of the environment instances (Sec. II): int32 [E], caller
 * env order, to out (out_on_device != 0: device pointer, enqueued; 0: host,
 * synchronous).  Bits: MG_FLAG_NONFINITE -- the state went non-finite in a
 * step (mg_step, mg_step_plain, mg_rollout), the env is frozen;
 * MG_FLAG_NOT_SPD -- the parameters of the last reset give a mass matrix that
 * is not positive definite, the env is frozen.  A Gym task step that restarts
 * an env clears its MG_FLAG_NONFINITE (and re-derives MG_FLAG_NOT_SPD when it
 * restarts with new multipliers).  NULL out: MG_ERR_INVALID. */
#define MG_FLAG_NONFINITE 1
#define MG_FLAG_NOT_SPD 2
mg_status mg_get_flags(mg_sim* sim, int32_t* out, int32_t out_on_device);

/* Bounds-checked debug build (not a passage of the paper: a checking aid).
 * The same sources built with -DMG_DEBUG give libmg_debug.so, with the same
 * entry points and results.  Its kernels check the indices each lane
 * addresses against the bounds of the buffers (a class segment within the
 * padded rows, caller columns within [0, n_envs), internal columns, tick-list
 * entries, page columns within their request's arrays); a failed check sets
 * its bit in a device word and that lane does nothing further, so it never
 * accesses memory out of bounds.  Bits: MG_DBG_SEGMENT, MG_DBG_COLUMN,
 * MG_DBG_INTERNAL, MG_DBG_LIST, MG_DBG_PAGE.
 * mg_debug_build: 1 in the debug build, 0 in the release build.
 * mg_debug_word: waits for the sim's stream, then stores the word in *word
 *   and zeroes it when clear != 0; the release build always stores 0.
 *   NULL word: MG_ERR_INVALID.
 * Test hook of the debug build: MG_DEBUG_SHRINK=k in the environment when a
 * sim is created makes its kernels treat caller columns >= n_envs - k as out
 * of bounds (those envs are skipped, and MG_DBG_COLUMN is set). */
#define MG_DBG_SEGMENT 1
#define MG_DBG_COLUMN 2
#define MG_DBG_INTERNAL 4
#define MG_DBG_LIST 8
#define MG_DBG_PAGE 16
int32_t mg_debug_build(void);
mg_status mg_debug_word(mg_sim* sim, uint32_t* word, int32_t clear);

/* Advances every env by n_ctrl control steps in ONE fused launch per class:
 * each control step reads one throttle frame, holds it for `substeps` RK4
 * sub-steps, and the state stays in registers across all n_ctrl * substeps
 * sub-steps (Sec. II: several sub-simulation steps per simulation step).
 *   actions  device [n_ctrl][N_max][E] throttles (rows >= a class's n_thr are ignored)
 *   targets  device [3][E] station-keeping targets for the statistics, or NULL (origin)
 *   traj     device [n_ctrl][D][E] state after each control step, or NULL
 *   stats    device double [n_ctrl][4] per control step, over envs that are
 *            not frozen: sum and max of |p - target| (the Task-1 error of
 *            Eq. (4)), sum of kinetic energy 1/2 nu^T M nu; and the number of
 *            frozen envs.  Deterministic (fixed-order two-pass reduction).  Or
 *            NULL.
 * Frozen envs: an env with a status flag set (mg_get_flags) is not stepped:
 * its state, and its traj rows, stay as they are.  An env whose state is not
 * finite at the end of a launch keeps the state it had when that launch began
 * -- with one control step per launch (mg_rollout, mg_step with n_ctrl = 1)
 * its last finite state -- and gets MG_FLAG_NONFINITE, so it is frozen from
 * the next launch on until mg_reset or mg_set_state gives it a new state; the
 * traj rows that launch wrote keep the non-finite values.  The other envs are
 * not affected.  The
 * split scheme (mg_step_split), the adjoint and the server neither read nor
 * set the flags: there a non-finite state propagates NaN. */
mg_status mg_step(mg_sim* sim, const float* actions, int32_t n_ctrl, const float* targets,
                  float* traj, double* stats);
/* The sub-simulation steps of Sec. II (the paragraph after Eq. (1)) taken one
 * per launch, as an engine that updates the dynamics once per sub-step does:
 * the same discrete map as mg_step, computed by the plain kernel, one launch
 * per RK4 sub-step per class, state round-tripping HBM between launches.  The
 * thruster lag states advance by the one-sub-step lag factor per launch
 * instead of its S-th power once per control step, so results agree with
 * mg_step to rounding, not bitwise. */
mg_status mg_step_plain(mg_sim* sim, const float* actions, int32_t n_ctrl, const float* targets,
                        float* traj, double* stats);
/* A sequence of T Gym-style steps (Sec. III) of every env with its
 * throttles (Eq. (3)) given up front, each of `substeps` sub-steps (Sec. II):
 * T control steps as T launches per class (plain != 0: T * substeps
 * launches), replayed from a HIP graph that is captured on first use and
 * cached for this exact argument tuple (at most 64 tuples per sim; the 65th
 * empties the cache, after waiting for the sim's stream).  Arguments as
 * mg_step with n_ctrl = T. */
mg_status mg_rollout(mg_sim* sim, const float* actions, int32_t T, const float* targets,
                     float* traj, double* stats, int32_t plain);
/* Reads back eta and nu of Eq. (1) (Sec. II) with the thruster states: copies
 * the state [D][E], caller env order, to out.  out_on_device != 0: device
 * pointer, enqueued; 0: host pointer, synchronous (waits for the stream).
 * NULL out: MG_ERR_INVALID. */
mg_status mg_get_state(mg_sim* sim, float* out, int32_t out_on_device);
/* Reads back the randomised physical parameters (Sec. II, component 1):
 * copies the absolute parameters [23][E], same rules as mg_get_state. */
mg_status mg_get_params(mg_sim* sim, float* out, int32_t out_on_device);
/* Simulation and learner share one GPU with few host transfers (Sec. III), so
 * every call above is stream-ordered; this is the host's wait: it blocks until
 * the sim's stream is idle and returns MG_ERR_DEVICE if queued work failed. */
mg_status mg_synchronize(mg_sim* sim);

/* The split integration that Sec. II describes, as a variant of mg_step: a
 * physics engine advances the rigid body (M_RB, C_RB, g_RB) by semi-implicit
 * Euler while the hydrodynamic wrench -M_A a_prev - C_A nu - D nu - g_A,
 * computed from the current state, acts on it as an external force; a_prev
 * is the env's rigid-body acceleration of its previous sub-step (kept by the
 * sim, 0 after mg_reset).  Per sub-step: nu += dt a, p += dt R(q) v with the
 * new v, q += dt/2 q (x) (0, omega) with the new omega then q /= |q|, thruster
 * lag by explicit Euler.  First order, and unstable on any axis whose added
 * mass exceeds its rigid-body inertia (the lagged term grows by M_A / M_RB per
 * sub-step).  Arguments as mg_step (no statistics). */
mg_status mg_step_split(mg_sim* sim, const float* actions, int32_t n_ctrl, float* traj);

/* ---- Gym-style tasks (Sec. III) ------------------------------------------------------
 * The four control tasks of Sec. III as vectorised environments: station
 * keeping and circle, helix and lemniscate tracking.  A task step is one
 * control step (as mg_step with n_ctrl = 1) followed, in the same launch, by
 * the task epilogue: the episode counter advances, the position error of
 * Eq. (4) is taken against the reference at the new episode time, an episode
 * ends terminated (done 1: non-finite state, or error above max_error > 0) or
 * truncated (done 2: episode_steps reached) and restarts at once, and the
 * observation of Eq. (2) is written.  The epilogue computes in FP64 from the
 * FP32 state.
 *
 * mg_task
 *   task           MG_TASK_STATION / CIRCLE / HELIX / LEMNISCATE
 *   lookahead      m, reference points in a tracking observation (1..16)
 *   radius         R (m); omega: rate of the curve parameter s = omega t + phase (rad/s)
 *   climb_rate     helix vertical rate (m/s along NED z)
 *   lookahead_dt   time between look-ahead points (s); <= 0: one control step
 *   episode_steps  control steps per episode (>= 1)
 *   max_error      error bound (m) that terminates an episode; 0: none
 * Reference points (t: seconds since the env's episode began):
 *   station    the env's centre; heading: its target yaw
 *   circle     c + R (cos s, sin s, 0); helix: the circle + (0, 0, climb_rate t)
 *   lemniscate c + R (cos s, sin s cos s, 0) / (1 + sin^2 s)  (Bernoulli)
 *   the reference attitude is level, headed along the horizontal reference velocity
 * Observation (caller layout [obs_dim][E]):
 *   station  [p - c, roll, pitch, wrap(yaw - target yaw), nu]          12 rows
 *   tracking for i = 1..m: [p - p_r(t + i dl), roll, pitch,
 *            wrap(yaw - heading_r(t + i dl))], then nu                  6 m + 6 rows
 *   NED position errors, ZYX Euler angles, angles in (-pi, pi].
 */
#define MG_TASK_STATION 0
#define MG_TASK_CIRCLE 1
#define MG_TASK_HELIX 2
#define MG_TASK_LEMNISCATE 3
#define MG_MAX_LOOKAHEAD 16

typedef struct {
  int32_t task, lookahead;
  double radius, omega, climb_rate, lookahead_dt;
  int32_t episode_steps, reserved;
  double max_error;
} mg_task;

/* Sets the task and each env's centre (device [3][E]), curve phase (device
 * [E]) and target yaw (device [E], or NULL: 0); every episode counter starts
 * at 0.  mg_reset also zeroes the counters of the envs whose state it
 * resets.  Copies the inputs (stream-ordered). */
mg_status mg_task_configure(mg_sim* sim, const mg_task* task, const float* center,
                            const float* phase, const float* yaw);
/* Observation rows: 12 (station keeping), 6 m + 6 (tracking); 0 if no task. */
int32_t mg_task_obs_dim(const mg_sim* sim);
/* Writes the observation of the current states to device obs [obs_dim][E]. */
mg_status mg_task_observe(mg_sim* sim, float* obs);
/* One Gym step of every env.
 *   actions      device [N_max][E] throttles of this control step
 *   obs          device [obs_dim][E] (written): after the step, or of the new
 *                episode where one ended
 *   err          device [E] position error of Eq. (4) after the step, or NULL
 *   done         device int32 [E]: 0 running, 1 terminated, 2 truncated, or NULL
 *   reset_state  device [D][E] states an ended episode restarts from, or NULL
 *                (at rest at the origin, identity attitude, no thrust)
 *   reset_mult   device [23][E] parameter multipliers an ended episode
 *                restarts with (refactorised as by mg_reset), or NULL (kept) */
mg_status mg_task_step(mg_sim* sim, const float* actions, float* obs, float* err, int32_t* done,
                       const float* reset_state, const float* reset_mult);
/* Copies the episode counters (control steps since each env's episode began)
 * to device int32 out [E]. */
mg_status mg_task_counters(mg_sim* sim, int32_t* out);

/* ---- discrete adjoint of a rollout -------------------------------------------------
 * The reverse mode of the exact discrete map mg_step computes (RK4 stages,
 * quaternion renormalisation, thruster lag and clamp), for gradient-based use
 * of the parallel environments of Sec. II.  Gradients are taken with respect
 * to the throttles, the initial state and the hydrodynamic parameters theta =
 * (M_A(6), D_L(6), D_Q(6), B) in absolute units (rows 4..22 of the 23-row
 * parameter layout); the sim's current parameters are used.
 *
 * mg_adj_forward: T control steps from the sim's current state (which it
 *   advances), one launch per class, storing the state before every
 *   ckpt_every-th control step.
 *   actions  device [T][N_max][E]
 *   ckpt     device [ceil(T / ckpt_every)][D][E]  (written)
 *   traj     device [T][D][E] state after each control step, or NULL
 * mg_adj_backward: given dL/d traj, recomputes each segment of ckpt_every
 *   control steps from its checkpoint and sweeps it backwards.  With one
 *   sub-step per control step and the forward's trajectory given (traj), the
 *   input of every step is already there (the row before it; ckpt for the
 *   first), so nothing is recomputed and no scratch is used.  Otherwise the sub-step
 *   states it linearises about are held in a scratch buffer the sim owns and
 *   keeps until mg_destroy: the whole rollout's (T * substeps * D * E floats)
 *   when that fits in 4 GiB, there is more than one segment and the allocation
 *   succeeds, every segment then recomputed at once before the sweep;
 *   otherwise one segment's (ckpt_every * substeps * D * E floats), recomputed
 *   just before its sweep.  The gradients are the same, bitwise, either way.
 *   MG_ERR_OOM only when the segment-sized buffer cannot be allocated.
 *   ckpt, actions  as written / read by mg_adj_forward with the same T, ckpt_every
 *   traj      device [T][D][E] the trajectory that forward wrote, unchanged, or
 *             NULL (used as above, else ignored); the gradients are the same,
 *             bitwise, with or without it
 *   dL_dtraj  device [T][D][E]
 *   dL_dact   device [T][N_max][E]  (written; rows >= a class's n_thr are 0,
 *             and so is the derivative of a clamped throttle)
 *   dL_dtheta device [19][E]        (written)
 *   dL_dx0    device [D][E] or NULL (written) */
mg_status mg_adj_forward(mg_sim* sim, const float* actions, int32_t T, int32_t ckpt_every,
                         float* ckpt, float* traj);
mg_status mg_adj_backward(mg_sim* sim, const float* ckpt, const float* traj,
                          const float* actions, int32_t T, int32_t ckpt_every,
                          const float* dL_dtraj, float* dL_dact, float* dL_dtheta,
                          float* dL_dx0);

/* mg_adj_backward for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving or training loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results (bitwise) as
 * mg_adj_backward, but the sub-step states it recomputes go to a static
 * scratch array of MG_NOALLOC_SCRATCH_BYTES that the library holds on every
 * device it runs on until the process ends; the call itself allocates
 * nothing.  The whole rollout's states are used when there is more than one
 * segment and T * substeps * D * E_pad floats fit (E_pad: the env count padded
 * per class to 256), else one segment's, ckpt_every * substeps * D * E_pad
 * floats (min(T, ckpt_every) for T < ckpt_every); a segment beyond the scratch
 * returns MG_ERR_INVALID with nothing done.  The scratch is shared by every
 * sim on the device and keeps the last call's contents (every float read is
 * first written by the same call): calls that overlap on one device, from any
 * sim or stream, race and must be ordered by the caller.  MG_ERR_DEVICE if the
 * scratch was not set up (mg_create looks it up once per device). */
#define MG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
mg_status mg_adj_backward_noalloc(mg_sim* sim, const float* ckpt, const float* traj,
                                  const float* actions, int32_t T, int32_t ckpt_every,
                                  const float* dL_dtraj, float* dL_dact, float* dL_dtheta,
                                  float* dL_dx0);

/* ---- serving loop -------------------------------------------------------------------
 * Serves step and rollout requests of uneven env counts from many client
 * threads on one GPU: the parallel environments of Sec. II, batched across
 * requests.  Continuous batching: a scheduler thread admits queued requests
 * FIFO whenever their pages (64 envs of one class each) fit under the memory
 * cap, keeps their states on the device, and advances every admitted request
 * by up to steps_per_tick control steps per tick with one launch over the
 * pages of all vehicle classes; a request that arrives while others run joins
 * at the next tick, and a finished one frees its pages at once.  Each env goes
 * through exactly the arithmetic of mg_step, so a request's result does not
 * depend on what else is in flight.
 *
 * mg_server_config
 *   classes, n_classes, dt_sub, substeps, device  as in mg_config
 *   mem_cap_bytes  page memory cap (> 0), or 0 to use mem_fraction
 *   mem_fraction   cap as a fraction of the device memory (0 -> 0.8)
 *   fifo_plain     1: baseline mode -- one request at a time, plain kernel
 *                  (one launch per sub-step); same results
 *   max_queue      bound of the admission queue (0 -> 65536)
 *   reserve_bytes  page memory (>= 0) to create at start (at most the cap),
 *                  with pinned staging for up to 4096 pages joining or
 *                  leaving per tick, 16 pinned result buffers of up to 16 MB
 *                  and a tick list for every reserved page, so that serving
 *                  within it allocates nothing: joins and retirements beyond
 *                  a tick's staging wait for a later tick instead (a request
 *                  larger than the staging alone still grows it); 0: pages
 *                  are created on demand in slabs of 1024 and staging grows as
 *                  needed.  Creation fails with MG_ERR_OOM if the reservation
 *                  cannot be had.
 *   steps_per_tick most control steps (0 -> 1, at most 64) a page advances per
 *                  tick: each active request advances min(steps_per_tick,
 *                  steps it has left), its states held in registers across
 *                  them.  More steps per tick cut the host's per-tick cost for
 *                  long rollouts (a 64-step request needs 64 / steps_per_tick
 *                  ticks); a request that arrives joins at the next tick, which
 *                  then lasts as long as its longest page's steps.  Results do
 *                  not depend on it.  Must be 0 or 1 with fifo_plain.
 * mg_request (everything the client passes stays owned by the client and
 * must stay valid until the request completes)
 *   n_envs, n_steps  env count (>= 1) and control steps (>= 1; 1 = a step request)
 *   env_class        host [n_envs] class per env, or NULL (all class 0); copied at submit
 *   x0               device [D][ld] initial states (first n_envs columns)
 *   param_mult       device [23][ld] parameter multipliers, or NULL (nominal)
 *   actions          device [n_steps][N_max][ld] throttles, or NULL with
 *                    actions_from_seed
 *   actions_from_seed 1: the throttles are generated on the device from
 *                    action_seed instead of read (actions is ignored): throttle
 *                    i of env e (0-based in the request) at control step t is
 *                    2 u - 1, u = (z >> 40) 2^-24, where z is output number
 *                    k = (t N_max + i) n_envs + e (0-based) of the SplitMix64
 *                    generator seeded with action_seed, i.e.
 *                    z = mix(action_seed + (k + 1) 0x9E3779B97F4A7C15) with
 *                    mix: z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
 *                    z *= 0x94D049BB133111EB; z ^= z >> 31 (Steele, Lea and
 *                    Flood, OOPSLA 2014).  U[-1, 1) on a 2^-23 grid, exact in
 *                    FP32.  0: read from actions.
 *   ld               column stride of x0, param_mult and actions (>= n_envs)
 *   out              host [D][n_envs]: the final states, written before completion
 *   arrival_ns       arrival stamp on the mg_clock_ns() clock, or 0 (= at submit;
 *                    a stamp later than the submission is replaced by it);
 *                    latency is measured from it to the moment out is written */
typedef struct mg_server mg_server;

typedef struct {
  uint32_t abi_version;
  int32_t n_classes;
  const mg_vehicle* classes;
  double dt_sub;
  int32_t substeps;
  int32_t device;
  int64_t mem_cap_bytes;
  double mem_fraction;
  int32_t fifo_plain;
  int32_t max_queue;
  int64_t reserve_bytes;
  int32_t steps_per_tick;
  int32_t reserved;
} mg_server_config;

typedef struct {
  int64_t n_envs;
  int32_t n_steps;
  int32_t actions_from_seed;
  const int32_t* env_class;
  const float* x0;
  const float* param_mult;
  const float* actions;
  int64_t ld;
  float* out;
  uint64_t arrival_ns;
  uint64_t action_seed;
} mg_request;

/* Server counters: requests completed / rejected, ticks issued, env control
 * steps done, envs active now and at most, requests queued now, the page cap
 * and pages created; host time spent issuing ticks and blocked waiting for the
 * GPU (ns, summed); mean and max time from arrival to admission (ns); the
 * longest host time spent issuing one tick (ns); how many times a staging
 * buffer had to grow (each growth allocates); with reserve_bytes, how many
 * times a join waited a tick because the tick's join staging was full, and how
 * many finished requests waited a tick to retire because the tick's result
 * staging was full (a reserved server allocates nothing for a request that
 * fits its staging alone). */
typedef struct {
  int64_t completed, rejected, ticks, env_steps, active_envs, max_active_envs, queued;
  int64_t cap_pages, created_pages;
  int64_t issue_ns, wait_ns, mean_queue_ns, max_queue_ns;
  int64_t max_issue_ns, grow_events, held_joins, deferred_retires;
} mg_server_stats;

/* The server's clock (std::chrono::steady_clock, ns): the time base of arrival stamps
 * and latencies (plumbing, no passage of the paper). */
uint64_t mg_clock_ns(void);
/* Starts the scheduler thread; page memory is taken in slabs as needed up to the cap. */
mg_status mg_server_create(const mg_server_config* cfg, mg_server** out);
/* Thread-safe.  MG_ERR_INVALID for a malformed request or one whose pages exceed
 * the whole cap (counted as rejected); MG_ERR_BUSY if the queue is full. */
mg_status mg_server_submit(mg_server* srv, const mg_request* req, uint64_t* ticket);
/* Waits up to timeout_us (< 0: forever; 0: a poll that returns at once) for a
 * ticket; MG_OK once its result is in
 * out (the ticket is then consumed and *latency_s, if not NULL, receives
 * arrival-to-completion seconds), MG_ERR_BUSY on timeout, MG_ERR_INVALID for an
 * unknown or already consumed ticket (also for a second thread waiting on a
 * ticket that another waiter consumed meanwhile), MG_ERR_DEVICE if the server
 * failed before the request completed: a failed tick fails every request in
 * flight or queued, and every later submit.  Test hook: with the environment
 * variable MG_SERVER_FAIL_TICK=n set when the server is created, the scheduler
 * treats the completion of its n-th tick (n >= 1) as a device error, without
 * any fault on the GPU. */
mg_status mg_server_wait(mg_server* srv, uint64_t ticket, int64_t timeout_us, double* latency_s);
/* Thread-safe.  Cancels a request that has not completed: a queued one leaves
 * the queue at once, an admitted one is retired at the scheduler's next tick
 * without its states being delivered, its pages freed; either then completes
 * with MG_ERR_CANCELLED (mg_server_wait).  A request that has already done
 * its last control step completes normally instead.  MG_OK when the
 * cancellation is registered, MG_ERR_INVALID for an unknown or completed
 * ticket. */
mg_status mg_server_cancel(mg_server* srv, uint64_t ticket);
mg_status mg_server_get_stats(const mg_server* srv, mg_server_stats* out);

/* The server's failed-check word of the debug build (mg_debug_word); read it
 * while no request is in flight.  Release build: 0.  NULL srv or word:
 * MG_ERR_INVALID. */
mg_status mg_server_debug_word(mg_server* srv, uint32_t* word, int32_t clear);
const char* mg_server_last_error(const mg_server* srv);
/* Stops accepting requests, finishes every request already submitted, joins
 * the scheduler and frees everything; NULL is ignored. */
void mg_server_destroy(mg_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* MG_H */
