"""Benchmark of the batched Fossen RK4 step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-plain]

Workload (one "step" = one episode of the hot path over one batch):
  1,048,576 envs, half BlueROV2 (6 thrusters) and half BlueROV2 Heavy
  (8 thrusters), FP32, +-20 % uniform parameter randomisation, quadratic
  throttle map with a 0.05 s thruster lag; each step resets every env
  (parameters + per-env factorisation of M = M_RB + M_A), then runs 200
  control steps, each one fused launch per class of 16 RK4 sub-steps of 5 ms
  with the episode statistics, replayed from a HIP graph.  Actions (6.7 GB),
  initial states and multipliers are generated once, seeded, and are resident
  in HBM before timing starts.

Prints one JSON line.  `value` is env-steps/s where an env-step is one RK4
sub-step of one environment (one Fossen RK4 step).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/s of batched Fossen RK4 step at 1M envs; served p50/p99 latency"
PEAK_FP32_VALU = 157.3e12      # MI355X published FP32 vector peak (packed)
PEAK_HBM = 8.0e12
# Algorithmic work of one env-substep for the roofline: the flops a structured
# formulation of the RK4 step needs (four right-hand sides of ~250-280 flops,
# the RK4 combination ~280, the renormalisation ~15; FMA = 2), ~1.35 kflop, and
# the bytes the plain per-sub-step kernel must move (state in and out, one
# throttle frame, the 23 randomised parameters).
ALGO_FLOPS_PER_ENV_SUBSTEP = 1350.0


def substep_flops(n_thr, lag, substeps):
    """Flops of one env-substep as the kernel formulates it (FMA = 2, one per add/mul):
    four right-hand sides up to the residual tau - C nu - D nu - g given the momentum
    M nu (130 each), the RK4 stages and combination of the kinematic rows (73), of the
    velocity rows through the pre-scaled inverse (h/2) M^-1 (122) and of the carried
    momentum (48), the quaternion renormalisation (12) and, with a thruster lag, the
    closed-form lag stage wrenches and the carried lag wrench (48); plus, per control
    step, the throttle map, the command wrench, the lag wrench, the end-of-control-step
    lag states and the momentum (29 N + 2; 14 N + 8 without lag) spread over the
    sub-steps."""
    core = 4 * 130 + 73 + 122 + 48 + 12
    lag_part = 48 if lag else 0
    per_ctrl = (29 * n_thr + 2) if lag else (14 * n_thr + 8)
    return core + lag_part + per_ctrl / substeps


def split_substep_flops(n_thr, lag, substeps):
    """Flops of one env-substep of the split scheme as its kernel formulates it (FMA = 2):
    the momentum M nu (14), the residual tau - C nu - D nu - g without the kinematic rows
    (83: the shared right-hand-side code's 130 less the 47 of the kinematic rows, which
    the split update does not use and the compiler drops), the lagged added-mass term
    (12), M_RB^-1 applied to the residual (14), the velocity, position and quaternion
    updates (12 + 36 + 28), the renormalisation (12) and, with a thruster lag, the lag
    wrench B (f - f_cmd) added to the command wrench and the lag-state update (16 N);
    plus, per control step, the throttle map and the command wrench (14 N - 6) spread
    over the sub-steps."""
    core = 14 + 83 + 12 + 14 + 12 + 36 + 28 + 12
    return core + (16 * n_thr if lag else 0) + (14 * n_thr - 6) / substeps


def progress(msg):
    """One line on stderr as each stage of the run ends (the JSON line goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def fused_algo_bytes(n_thr, lag):
    """Algorithmic HBM bytes of one env in one fused launch (one control step of S
    sub-steps): state read once and written once, one throttle frame, the 23 randomised
    parameters -- the plain kernel's per-sub-step bytes, moved once per control step."""
    return plain_bytes(n_thr, lag)


def plain_bytes(n_thr, lag):
    """Algorithmic HBM bytes of one env-substep in the plain kernel: state read+write,
    the throttle frame, the 23 randomised parameters."""
    D = 13 + (n_thr if lag else 0)
    return 4 * (2 * D + n_thr + 23)


def source_hash(files):
    """Hash of the named files of paper_2410_14117_amd/csrc (a profile summary records the
    hash of the sources its kernels are compiled from)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2410_14117_amd", "csrc")
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


STEP_SOURCES = ("kernels_step.hip", "fossen_device.h", "mg_internal.h")
ADJOINT_SOURCES = ("kernels_adjoint.hip", "fossen_adjoint.h", "fossen_device.h", "mg_internal.h")
SERVE_SOURCES = ("kernels_serve.hip", "server.hip", "fossen_device.h", "mg_internal.h")
SPLIT_TASK_SOURCES = ("kernels_split.hip", "kernels_task.hip", "fossen_device.h", "mg_internal.h")


def kernel_source_hash():
    """Hash of the sources the step kernels are compiled from (their traffic and counters
    in profiles/ hold only while these are unchanged)."""
    return source_hash(STEP_SOURCES)


def load_traffic(kernel_key):
    """HBM traffic per launch from the committed rocprofv3 --pmc summary, if it was taken
    on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get(kernel_key)


def cpu_baseline(n_envs=1 << 16, n_ctrl=200, n_envs_1t=1024):
    """The FP64 oracle as it stands, on a bounded sample of the same workload (2^16 envs on
    all host threads, about 10 s on 16 threads; and 1024 envs on one thread)."""
    from oracle import oracle
    from workloads import (BLUEROV2, BLUEROV2_HEAVY, CONFIGS, vehicle_variant, initial_state,
                           actions, param_multipliers, env_classes)
    c = CONFIGS["c3"]
    classes = [vehicle_variant(BLUEROV2, thr_map=1, thr_tau=0.05),
               vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)]
    cls = env_classes(n_envs, "halves")
    x0 = initial_state(n_envs, 21, c.seed_base + 2)
    act = actions(n_ctrl, 8, n_envs, c.seed_base + 3)
    mult = param_multipliers(n_envs, c.rho, c.seed_base + 1)
    oracle.build()
    threads = oracle.lib().or_max_threads()
    t0 = time.perf_counter()
    oracle.rollout(classes, x0, act, c.substeps, c.dt_sub, env_class=cls, mult=mult,
                   want_stats=True, nthreads=threads)
    dt = time.perf_counter() - t0
    # one thread, on the first 512 envs of each class
    sel = np.r_[0:n_envs_1t // 2, n_envs // 2:n_envs // 2 + n_envs_1t // 2]
    t0 = time.perf_counter()
    oracle.rollout(classes, np.ascontiguousarray(x0[:, sel]),
                   np.ascontiguousarray(act[:, :, sel]), c.substeps, c.dt_sub,
                   env_class=cls[sel], mult=np.ascontiguousarray(mult[:, sel]), want_stats=True,
                   nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": n_envs * n_ctrl * c.substeps / dt, "unit": "env-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_envs} envs (half BlueROV2, half Heavy) x {n_ctrl} control steps x "
                      f"{c.substeps} RK4 sub-steps, FP64, with statistics; {dt:.2f} s on "
                      f"{threads} threads",
            "value_1_thread": n_envs_1t * n_ctrl * c.substeps / dt1,
            "sample_1_thread": f"{n_envs_1t} of those envs (half of each class), same steps, "
                               f"one thread; {dt1:.2f} s",
            "other_workloads": cpu_other_workloads(threads)}


def cpu_other_workloads(threads):
    """The oracle on the other workloads, in full where that takes seconds: 64 BlueROV2
    envs x 1000 steps (nominal, linear map); 4096 Heavy envs x 1000 control steps x 4
    sub-steps (+-20 %, quadratic map, lag); the 8192-env, 64-step tracking-loss forward;
    and its dual-number gradient (throttles, 19 parameters, x0) on 16 envs."""
    from oracle import oracle
    from workloads import (BLUEROV2, BLUEROV2_HEAVY, CONFIGS, vehicle_variant, initial_state,
                           actions, param_multipliers, circle_waypoints)
    out = {}
    c1 = CONFIGS["c1"]
    x0 = initial_state(c1.n_envs, 13, c1.seed_base + 2)
    act = actions(c1.n_ctrl, 6, c1.n_envs, c1.seed_base + 3)
    t0 = time.perf_counter()
    oracle.rollout(BLUEROV2, x0, act, c1.substeps, c1.dt_sub, want_stats=True, nthreads=threads)
    dt = time.perf_counter() - t0
    out["c1_full"] = {"env_steps_per_s": c1.n_envs * c1.n_ctrl * c1.substeps / dt, "s": dt,
                      "workload": "64 BlueROV2 envs x 1000 steps of 10 ms, nominal, linear map"}
    c2 = CONFIGS["c2"]
    heavy = vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)
    x0 = initial_state(c2.n_envs, 21, c2.seed_base + 2)
    act = actions(c2.n_ctrl, 8, c2.n_envs, c2.seed_base + 3)
    mult = param_multipliers(c2.n_envs, c2.rho, c2.seed_base + 1)
    t0 = time.perf_counter()
    oracle.rollout(heavy, x0, act, c2.substeps, c2.dt_sub, mult=mult, want_stats=True,
                   nthreads=threads)
    dt = time.perf_counter() - t0
    out["c2_full"] = {"env_steps_per_s": c2.n_envs * c2.n_ctrl * c2.substeps / dt, "s": dt,
                      "workload": "4096 Heavy envs x 1000 control steps x 4 sub-steps of 5 ms, "
                                  "+-20 %, quadratic map, 0.05 s lag"}
    c4 = CONFIGS["c4"]
    E, T = c4.n_envs, c4.n_ctrl
    x0 = initial_state(E, 13, c4.seed_base + 2)
    act = actions(T, 6, E, c4.seed_base + 3)
    pref, qref = circle_waypoints(T, E, c4.dt_sub, c4.seed_base + 4, omega=c4.extra["omega"])
    t0 = time.perf_counter()
    oracle.track_loss(BLUEROV2, x0, act, c4.substeps, c4.dt_sub, pref, qref, nthreads=threads)
    dt_f = time.perf_counter() - t0
    sub = slice(0, 16)
    t0 = time.perf_counter()
    oracle.track_loss_grad(BLUEROV2, np.ascontiguousarray(x0[:, sub]),
                           np.ascontiguousarray(act[:, :, sub]), c4.substeps, c4.dt_sub,
                           np.ascontiguousarray(pref[:, :, sub]),
                           np.ascontiguousarray(qref[:, :, sub]), want_x0=True, nthreads=threads)
    dt_g = time.perf_counter() - t0
    out["c4_forward"] = {"ms": dt_f * 1e3, "env_steps_per_s": E * T / dt_f,
                         "workload": "8192 BlueROV2 envs x 64 steps of 10 ms with the tracking "
                                     "loss"}
    out["c4_dual_gradient_16_envs"] = {
        "ms": dt_g * 1e3, "gradients_per_s": 16 / dt_g,
        "workload": "forward-mode (dual number) gradient of the tracking loss w.r.t. 64 x 6 "
                    "throttles, 19 parameters and x0, envs 0-15"}
    return out


def bench_adjoint(torch, mg, reps=5, n_envs=None):
    """C4: 8192 BlueROV2 envs, 64 control steps of 10 ms, checkpoint every 8; forward with
    checkpoints and the trajectory (which the loss needs), backward (the reverse sweep,
    reading each step's input from the trajectory: one sub-step per control step), against
    the plain per-step launch."""
    from workloads import BLUEROV2, CONFIGS, initial_state, actions
    c = CONFIGS["c4"]
    E, T, K = n_envs or c.n_envs, c.n_ctrl, c.extra["ckpt_every"]
    dev = torch.device("cuda:0")
    x0 = torch.from_numpy(initial_state(E, 13, c.seed_base + 2)).to(dev)
    act = torch.from_numpy(actions(T, 6, E, c.seed_base + 3)).to(dev)
    g = torch.randn((T, 13, E), generator=torch.Generator(device=dev).manual_seed(4),
                    device=dev)
    sim = mg.Sim(BLUEROV2, E, c.dt_sub, c.substeps)
    traj = torch.empty((T, 13, E), device=dev)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(reps):
            fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    ckpt = [None]

    def fwd():
        sim.set_state(x0)
        ckpt[0], _ = sim.adj_forward(act, K, traj=traj)

    t_fwd = timed(fwd)
    t_bwd = timed(lambda: sim.adj_backward(ckpt[0], act, K, g, traj=traj))

    def plain():
        sim.set_state(x0)
        sim.rollout(act, plain=True)

    t_plain = timed(plain)
    sim.close()
    del traj, g, act, ckpt
    torch.cuda.empty_cache()
    return {"workload": f"{E} BlueROV2 envs, 64 control steps of 10 ms, checkpoint every 8, "
                        "gradients w.r.t. throttles, 19 hydrodynamic parameters and x0; the "
                        "backward reads each step's input from the forward's trajectory",
            "forward_ms": t_fwd, "backward_ms": t_bwd, "fwd_plus_bwd_ms": t_fwd + t_bwd,
            "cost_vs_forward": (t_fwd + t_bwd) / t_fwd,
            "plain_forward_ms": t_plain, "cost_vs_plain_forward": (t_fwd + t_bwd) / t_plain,
            "gradients_per_s": E / ((t_fwd + t_bwd) * 1e-3)}


def bench_serving(torch, mg, duration_s=30.0, fifo_plain=False, seed=5005, warmup_s=5.0,
                  reserve_bytes=2 << 30, steps_per_tick=1):
    """C5: 32 clients with Poisson arrivals (2000 req/s aggregate), env counts log-uniform in
    [16, 65536], half step requests (1 control step) and half rollouts (1..64 steps), mixed
    BlueROV2 / Heavy (+-20 % randomisation, 4 RK4 sub-steps of 5 ms per control step),
    initial states and multipliers resident on the device, throttles generated on the
    device from a per-request seed; latency = arrival -> final states in host memory.  The
    trace is replayed by 32 native client threads (one per client, libmg_clients.so), each
    submitting its own requests at their arrival times and waiting for them.  The server
    creates `reserve_bytes` of page memory at start, and a warm-up trace of `warmup_s`
    (another seed) runs first on it, so that the timed trace finds its pages and staging
    buffers allocated.  `steps_per_tick`: most control steps a request advances per tick."""
    from workloads import (BLUEROV2, BLUEROV2_HEAVY, CONFIGS, vehicle_variant, initial_state,
                           param_multipliers, env_classes)
    c = CONFIGS["c5"]
    classes = [vehicle_variant(BLUEROV2, thr_map=1, thr_tau=0.05),
               vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)]
    P, LMAX, D = 1 << 17, 64, 21
    dev = torch.device("cuda:0")
    cls = env_classes(P, "bernoulli", c.seed_base + 5)
    x0 = initial_state(P, D, c.seed_base + 2)
    x0[19:, cls == 0] = 0
    x0_d = torch.from_numpy(x0).to(dev)
    mult_d = torch.from_numpy(param_multipliers(P, c.rho, c.seed_base + 1)).to(dev)
    torch.cuda.synchronize()
    srv = mg.Server(classes, c.dt_sub, c.substeps, fifo_plain=fifo_plain,
                    reserve_bytes=reserve_bytes, steps_per_tick=steps_per_tick)
    n_clients, rate = c.extra["clients"], c.extra["rate"]

    def make_trace(seconds, trace_seed):
        # per client a Poisson stream of rate / n_clients
        rng = np.random.Generator(np.random.PCG64(trace_seed))
        trace = []
        for k in range(n_clients):
            t = 0.0
            while True:
                t += rng.exponential(n_clients / rate)
                if t > seconds:
                    break
                n = int(round(np.exp(rng.uniform(np.log(c.extra["env_lo"]),
                                                 np.log(c.extra["env_hi"])))))
                L = 1 if rng.random() < 0.5 else int(rng.integers(1, LMAX + 1))
                off = int(rng.integers(0, P - n + 1))
                trace.append((k, t, n, L, off, int(rng.integers(0, 2 ** 63))))
        trace.sort(key=lambda r: r[1])
        return trace

    def run(trace):
        # open loop: latency counts from the scheduled arrival.  The clients' result
        # buffers are allocated and touched before the trace starts, as a serving client
        # keeps them (fresh memory would add its page faults to the measured latency).
        sizes = [D * r[2] for r in trace]
        arena = np.ones(sum(sizes), np.float32)
        starts = np.concatenate([[0], np.cumsum(sizes)])
        reqs = [{"client": k, "at_ns": int(t * 1e9), "n_envs": n, "n_steps": L,
                 "x0_ptr": x0_d.data_ptr() + 4 * off, "ld": P,
                 "out": arena[starts[i]:starts[i + 1]].reshape(D, -1),
                 "env_class": cls[off:off + n], "mult_ptr": mult_d.data_ptr() + 4 * off,
                 "action_seed": aseed}
                for i, (k, t, n, L, off, aseed) in enumerate(trace)]
        status, lat, lag, t0 = srv.replay(reqs, n_clients)
        wall = (mg.Server.clock_ns() - t0) * 1e-9
        ok = status == 0
        env_steps = sum(r[2] * r[3] for r, o in zip(trace, ok) if o)
        # requests slower than 10 ms, grouped into episodes by arrival (gaps < 50 ms)
        slow = sorted((trace[i][1], float(lat[i])) for i in range(len(trace))
                      if ok[i] and lat[i] > 0.01)
        episodes = []
        for t, l in slow:
            if episodes and t - episodes[-1][1] < 0.05:
                e = episodes[-1]
                episodes[-1] = (e[0], t, e[2] + 1, max(e[3], l))
            else:
                episodes.append((t, t, 1, l))
        slow_summary = [{"from_s": round(a, 4), "to_s": round(b, 4), "requests": n,
                         "max_ms": round(m * 1e3, 2)} for a, b, n, m in episodes[:20]]
        return lat[ok], env_steps, wall, lag, int((~ok).sum()), slow_summary

    if warmup_s > 0:
        run(make_trace(warmup_s, seed + 1))
    s0 = srv.stats()
    trace = make_trace(duration_s, seed)
    lats, env_steps, wall, lags, failed, slow = run(trace)
    s1 = srv.stats()
    srv.close()
    ticks = max(1, s1["ticks"] - s0["ticks"])
    return {"mode": "fifo_plain_one_at_a_time" if fifo_plain else "continuous_batching",
            "clients": f"{n_clients} native client threads, each submitting its own Poisson "
                       "stream and waiting for its tickets",
            "actions": "generated on the device from a per-request SplitMix64 seed",
            "requests": len(trace), "completed": int(len(lats)), "failed": failed,
            "offered_req_per_s": len(trace) / duration_s, "trace_s": duration_s,
            "warmup_trace_s": warmup_s, "reserved_bytes": reserve_bytes,
            "steps_per_tick": steps_per_tick,
            "wall_s": wall, "req_per_s": len(lats) / wall,
            "env_control_steps_per_s": env_steps / wall,
            "env_steps_per_s": env_steps * c.substeps / wall,
            "p50_ms": float(np.percentile(lats, 50) * 1e3),
            "p99_ms": float(np.percentile(lats, 99) * 1e3),
            "p999_ms": float(np.percentile(lats, 99.9) * 1e3),
            "max_ms": float(lats.max() * 1e3),
            "max_active_envs": s1["max_active_envs"], "ticks": ticks,
            "host_issue_us_per_tick": (s1["issue_ns"] - s0["issue_ns"]) / ticks / 1e3,
            "host_blocked_us_per_tick": (s1["wait_ns"] - s0["wait_ns"]) / ticks / 1e3,
            "queue_wait_max_ms_incl_warmup": s1["max_queue_ns"] / 1e6,
            "max_tick_issue_ms_incl_warmup": s1["max_issue_ns"] / 1e6,
            "staging_growths": s1["grow_events"] - s0["grow_events"],
            "held_joins": s1["held_joins"] - s0["held_joins"],
            "deferred_retires": s1["deferred_retires"] - s0["deferred_retires"],
            "pages_created": s1["created_pages"] - s0["created_pages"],
            "slow_episodes": slow,
            "submit_lag_p50_ms": float(np.percentile(lags, 50) / 1e6),
            "submit_lag_p99_ms": float(np.percentile(lags, 99) / 1e6)}


def bench_task(torch, sim, act, x0, n_b, n_h, n_steps=60):
    """Gym-style circle tracking on the benchmark's envs: 4 look-ahead points in the
    observation (30 rows), episodes of 100 control steps with automatic reset, the error of
    Eq. (4) and the done flags; n_steps task steps (one launch per class each, issued from
    Python) against as many single-control-step mg_step calls issued the same way (the
    states drift apart between the passes; both advance the same envs by one control step
    per call)."""
    E, dev = sim.n_envs, x0.device
    g = torch.Generator(device="cpu").manual_seed(7007)
    center = torch.zeros((3, E), dtype=torch.float32, device=dev)
    phase = (torch.rand(E, generator=g) * 6.283185307179586).to(dev)
    task = {"task": "circle", "lookahead": 4, "radius": 2.0, "omega": 0.5, "episode_steps": 100}
    sim.reset(state=x0)
    sim.task_configure(task, center, phase)
    obs = torch.empty((sim.obs_dim, E), dtype=torch.float32, device=dev)
    err = torch.empty((E,), dtype=torch.float32, device=dev)
    done = torch.empty((E,), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        e0.record(stream)
        for t in range(n_steps):
            fn(t % act.shape[0])
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n_steps

    def task_fn(t):
        sim.task_step(act[t], obs, err, done, reset_state=x0)

    def step_fn(t):
        sim.step(act[t:t + 1])

    # both warmed up, then timed alternately twice, best of two each (the GPU's clock
    # settles during the first passes, which would otherwise penalise whichever runs first)
    for fn in (task_fn, step_fn):
        for t in range(3):
            fn(t)
    torch.cuda.synchronize()
    task_ms, step_ms = float("inf"), float("inf")
    for _ in range(2):
        task_ms = min(task_ms, timed(task_fn))
        step_ms = min(step_ms, timed(step_fn))
    S = sim.substeps
    flops = S * (n_b * substep_flops(6, True, S) + n_h * substep_flops(8, True, S))
    return {"workload": f"{E} envs (the benchmark's mix), circle tracking, m = 4 look-ahead "
                        "points, episodes of 100 control steps, automatic reset",
            "obs_rows": sim.obs_dim, "ms_per_task_step": task_ms,
            "ms_per_plain_control_step_call": step_ms,
            "epilogue_overhead": task_ms / step_ms - 1.0,
            "env_task_steps_per_s": E / (task_ms * 1e-3),
            "env_steps_per_s": E * S / (task_ms * 1e-3),
            "roofline": {"bound": "alu", "kernel": "k_task<6|8,lag>: the fused control step and "
                                                   "the task epilogue, both class launches",
                         "achieved": flops / (task_ms * 1e-3) / 1e12,
                         "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                         "frac": flops / (task_ms * 1e-3) / PEAK_FP32_VALU,
                         "counted": "the control step's flops (the fused step's tally); the "
                                    "epilogue's sincos, atan2 and FP64 work is not counted",
                         "epilogue_bytes_per_env": 4 * sim.obs_dim + 8 + 24}}


def bench_policy(torch, mg, n_envs, steps=100, warmup=10, horizon=16, graph=False):
    """Policy in the loop (the sampling side of the paper's PPO setup, Sec. III): BlueROV2
    Heavy envs on the circle task (m = 4 look-ahead points, 30 observation rows, episodes of
    100 control steps of 4 x 5 ms, automatic reset); per step an actor and a critic MLP
    (30-256-128-64, ELU; FP32, random init) read the observation, Gaussian actions are
    sampled and clamped, mg_task_step advances every env, and observation, action, reward
    (-error) and done go into a rollout buffer of `horizon` steps, all on the GPU.  The
    learner's update is not part of it.  graph=True captures the step once per rollout slot
    (policy, sampling, mg_task_step, buffer writes) in HIP graphs and replays them in turn."""
    from workloads import BLUEROV2_HEAVY, vehicle_variant, initial_state
    dev = torch.device("cuda:0")
    E, N = n_envs, 8
    heavy = vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)
    sim = mg.Sim(heavy, E, 0.005, 4)
    x0 = torch.from_numpy(initial_state(E, sim.state_dim, 9101)).to(dev)
    sim.reset(state=x0)
    g = torch.Generator(device="cpu").manual_seed(9102)
    sim.task_configure({"task": "circle", "lookahead": 4, "radius": 2.0, "omega": 0.5,
                        "episode_steps": 100},
                       (torch.randn((3, E), generator=g) * 0.3).to(dev),
                       (torch.rand(E, generator=g) * 6.283185307179586).to(dev))
    torch.manual_seed(9103)

    def mlp(n_out):
        return torch.nn.Sequential(torch.nn.Linear(sim.obs_dim, 256), torch.nn.ELU(),
                                   torch.nn.Linear(256, 128), torch.nn.ELU(),
                                   torch.nn.Linear(128, 64), torch.nn.ELU(),
                                   torch.nn.Linear(64, n_out)).to(dev)

    actor, critic = mlp(N), mlp(1)
    log_std = torch.full((N,), -1.0, device=dev)
    buf_obs = torch.empty((horizon, E, sim.obs_dim), device=dev)
    buf_act = torch.empty((horizon, E, N), device=dev)
    buf_val = torch.empty((horizon, E), device=dev)
    buf_rew = torch.empty((horizon, E), device=dev)
    buf_done = torch.empty((horizon, E), dtype=torch.int32, device=dev)
    err = torch.empty((E,), device=dev)
    done = torch.empty((E,), dtype=torch.int32, device=dev)
    # the observation ping-pongs between two buffers: step i reads obs_pair[i % 2]
    # and writes obs_pair[(i + 1) % 2] (horizon is even, so slot h fixes the roles)
    obs_pair = [sim.task_observe(), None]
    obs_pair[1] = torch.empty_like(obs_pair[0])

    def one(h):
        src, dst = obs_pair[h % 2], obs_pair[(h + 1) % 2]
        with torch.no_grad():
            o = src.t()
            buf_obs[h].copy_(o)
            mu = actor(o)
            a = (mu + torch.randn_like(mu) * log_std.exp()).clamp_(-1.0, 1.0)
            buf_act[h].copy_(a)
            buf_val[h].copy_(critic(o).squeeze(1))
            sim.task_step(a.t().contiguous(), dst, err, done, reset_state=x0)
            torch.neg(err, out=buf_rew[h])
            buf_done[h].copy_(done)

    if graph:
        # one graph per rollout slot, captured in slot order into one memory pool
        # and replayed in that order: the same work as the eager step
        s_side = torch.cuda.Stream()
        s_side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s_side):
            for h in range(4):
                one(h)
        torch.cuda.current_stream().wait_stream(s_side)
        torch.cuda.synchronize()
        pool = torch.cuda.graph_pool_handle()
        graphs = []
        for h in range(horizon):
            g_h = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g_h, pool=pool):
                one(h)
            graphs.append(g_h)
        run = lambda i: graphs[i % horizon].replay()      # noqa: E731
    else:
        run = lambda i: one(i % horizon)                    # noqa: E731
    for i in range(warmup):
        run(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(warmup, warmup + steps):
        run(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.close()
    return {"workload": f"{E} BlueROV2 Heavy envs, circle task (30 observation rows), actor + "
                        "critic MLP 30-256-128-64 (FP32), Gaussian actions, rollout buffer "
                        f"of {horizon} steps",
            "issued": "one HIP graph replay per step (one graph per rollout slot)" if graph
                      else "eagerly from Python",
            "n_envs": E, "steps": steps, "ms_per_step": wall * 1e3 / steps,
            "env_steps_per_s": E * steps / wall,
            "sim_seconds_per_wall_second": E * steps * 4 * 0.005 / wall}


def bench_split(torch, mg, classes, cls, act, x0, mult, n_ctrl=50):
    """The split scheme of Sec. II (mg_step_split) on the benchmark's envs: its rate, the
    share of envs that blow up (non-finite or |x| > 1e6) within n_ctrl control steps with
    the presets (heave and sway added mass above the vehicle mass) and with the added mass
    scaled by 0.4 (stable), and, for the latter, the position gap to the coupled RK4 step."""
    import copy
    E, dev = x0.shape[1], x0.device
    n_ctrl = min(n_ctrl, act.shape[0])
    n_b = int((cls == 0).sum())
    n_h = E - n_b
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {"workload": f"{E} envs (the benchmark's mix), {n_ctrl} control steps of 16 x 5 ms "
                       "in one launch per class"}
    for label, factor in (("presets", 1.0), ("added_mass_x0.4", 0.4)):
        cl = [copy.deepcopy(v) for v in classes]
        for v in cl:
            v["added_mass"] = [a * factor for a in v["added_mass"]]
        sim = mg.Sim(cl, E, 0.005, 16, env_class=cls)
        sim.reset(state=x0, param_mult=mult)
        sim.step_split(act[:2])
        torch.cuda.synchronize()
        sim.reset(state=x0, param_mult=mult)
        torch.cuda.synchronize()
        e0.record(stream)
        sim.step_split(act[:n_ctrl])
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        xs = sim.get_state()
        blown = (~torch.isfinite(xs).all(dim=0)) | (xs.abs().amax(dim=0) > 1e6)
        flops = n_ctrl * 16 * (n_b * split_substep_flops(6, True, 16) +
                               n_h * split_substep_flops(8, True, 16))
        res = {"env_steps_per_s": E * n_ctrl * 16 / (ms * 1e-3),
               "blown_share": float(blown.float().mean()),
               "roofline": {"bound": "alu", "kernel": "k_split<6|8,lag>, both class launches",
                            "achieved": flops / (ms * 1e-3) / 1e12,
                            "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                            "frac": flops / (ms * 1e-3) / PEAK_FP32_VALU,
                            "flops_per_env_substep": {
                                "bluerov2": split_substep_flops(6, True, 16),
                                "heavy": split_substep_flops(8, True, 16)}}}
        if factor != 1.0:
            sim.reset(state=x0, param_mult=mult)
            sim.step(act[:n_ctrl])
            gap = (xs[:3] - sim.get_state()[:3]).norm(dim=0)
            res["position_gap_to_rk4_m"] = {"median": float(gap.median()),
                                            "p99": float(torch.quantile(gap[:1 << 16], 0.99)),
                                            "max": float(gap.max())}
        sim.close()
        out[label] = res
    return out


def summarise_profile(root):
    """Summary of rocprofv3 CSV output under `root` (host-only, no GPU): per-kernel launch
    statistics from kernel_stats.csv; for the k_step launches of a kernel trace the union of
    their busy intervals per launch pair (the BlueROV2 and Heavy launches of one control or
    sub-step run concurrently, so the pair's wall time is the figure comparable with the
    bench's per-control-step time); per-kernel counter means from --pmc runs."""
    import csv
    import collections
    import glob
    out = []
    for f in sorted(glob.glob(os.path.join(root, "**", "*kernel_stats.csv"), recursive=True)):
        out.append(f"## {os.path.relpath(f, root)}")
        out.append("| kernel | calls | avg (us) | min (us) | max (us) | share |")
        out.append("|---|---|---|---|---|---|")
        for r in csv.DictReader(open(f)):
            out.append(f"| `{r['Name'][:100]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                       f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                       f"{float(r['Percentage']):.2f} % |")
    for f in sorted(glob.glob(os.path.join(root, "**", "*kernel_trace.csv"), recursive=True)):
        rows = list(csv.DictReader(open(f)))
        out.append(f"## {os.path.relpath(f, root)}")
        for label, plain in (("fused k_step", "false"), ("plain k_step", "true")):
            ivs = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in rows
                         if r["Kernel_Name"].startswith("void mg::k_step<")
                         and r["Kernel_Name"].split(",")[2].strip().startswith(plain))
            if not ivs:
                continue
            union, cs, ce = 0, None, None
            for a, b in ivs:
                if ce is None or a > ce:
                    union += 0 if ce is None else ce - cs
                    cs, ce = a, b
                else:
                    ce = max(ce, b)
            union += ce - cs
            mean = sum(b - a for a, b in ivs) / len(ivs)
            out.append(f"{label}: {len(ivs)} launches, mean launch {mean / 1e3:.2f} us, union of "
                       f"busy intervals {union / 1e3:.1f} us = {2 * union / len(ivs) / 1e3:.2f} us "
                       f"per launch pair")
    for f in sorted(glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True)):
        agg = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(f)):
            agg[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        out.append(f"## {os.path.relpath(f, root)}")
        out.append("| kernel | counter | dispatches | mean | min | max |")
        out.append("|---|---|---|---|---|---|")
        for k, cs_ in agg.items():
            for cname, v in cs_.items():
                out.append(f"| `{k[:80]}` | {cname} | {len(v)} | {sum(v) / len(v):.7g} | "
                           f"{min(v):.7g} | {max(v):.7g} |")
    return "\n".join(out)


def traffic_from_counters(root):
    """The content of profiles/traffic.json from the FETCH_SIZE and WRITE_SIZE --pmc runs
    under root (pmc_fetch/, pmc_write/; bench.py run with --calib-copy): per-dispatch means
    (KiB) of the fused and, when present, plain step launches of each class, scaled by what
    each counter reads for the 1 GiB device copy, in bytes; host-only."""
    import csv
    import collections
    import glob

    def load(sub, counter):
        vals = collections.defaultdict(list)
        for f in glob.glob(os.path.join(root, sub, "**", "*counter_collection.csv"),
                           recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    vals[r["Kernel_Name"]].append(float(r["Counter_Value"]))
        return vals

    fetch, write = load("pmc_fetch", "FETCH_SIZE"), load("pmc_write", "WRITE_SIZE")
    gib_kib = float(1 << 20)
    ff = gib_kib / max(fetch["__amd_rocclr_copyBuffer"])
    fw = gib_kib / max(write["__amd_rocclr_copyBuffer"])

    def per_launch(n, plain):
        k = f"void mg::k_step<{n}, true, {'true' if plain else 'false'}>(mg::StepArgs, mg::ClassConst)"
        if k not in fetch or k not in write:
            return None
        return 1024.0 * (ff * sum(fetch[k]) / len(fetch[k]) + fw * sum(write[k]) / len(write[k]))

    out = {"source_hash": kernel_source_hash(),
           "what": "HBM bytes from rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE runs (KiB "
                   "per dispatch, mean over the dispatches of each class), each scaled by what "
                   f"the same counter reads for a 1 GiB device copy (FETCH x{ff:.6f}, WRITE "
                   f"x{fw:.6f}); fused: both class launches of one control step (524,288 "
                   "BlueROV2 + 524,288 Heavy envs, 16 RK4 sub-steps); plain: both class "
                   "launches of one sub-step",
           "per_launch": {}, "fetch_factor": ff, "write_factor": fw}
    for label, n, plain in (("fused_bluerov2", 6, False), ("fused_heavy", 8, False),
                            ("plain_bluerov2", 6, True), ("plain_heavy", 8, True)):
        v = per_launch(n, plain)
        if v is not None:
            out["per_launch"][label] = v
    pl = out["per_launch"]
    if "fused_bluerov2" in pl and "fused_heavy" in pl:
        out["k_step_fused_control_step"] = pl["fused_bluerov2"] + pl["fused_heavy"]
    if "plain_bluerov2" in pl and "plain_heavy" in pl:
        out["k_step_plain_substep"] = pl["plain_bluerov2"] + pl["plain_heavy"]
    out["algorithmic_fused_control_step"] = (524288 * fused_algo_bytes(6, True) +
                                             524288 * fused_algo_bytes(8, True))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n-envs", type=int, default=1 << 20)
    ap.add_argument("--n-ctrl", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-task", action="store_true")
    ap.add_argument("--no-policy", action="store_true")
    ap.add_argument("--no-split", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="timed serving trace (after a --serve-warmup trace of another seed)")
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-aux-seconds", type=float, default=5.0,
                    help="timed trace of the one-step-per-tick comparison")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one device copy of 1 GiB (read 1 GiB, write 1 GiB) whose "
                         "FETCH_SIZE / WRITE_SIZE calibrate the counters of a --pmc run")
    ap.add_argument("--summarise-profile", metavar="DIR",
                    help="print a summary of the rocprofv3 CSV files under DIR and exit")
    ap.add_argument("--traffic-from", metavar="DIR",
                    help="write profiles/traffic.json from the FETCH_SIZE / WRITE_SIZE runs "
                         "under DIR (pmc_fetch/, pmc_write/) and exit")
    args = ap.parse_args()
    if args.summarise_profile:
        print(summarise_profile(args.summarise_profile))
        return
    if args.traffic_from:
        t = traffic_from_counters(args.traffic_from)
        with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
            json.dump(t, f, indent=1)
        print(json.dumps(t))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the environments are independent and this "
              "build runs no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2410_14117_amd import mg
    from workloads import (BLUEROV2, BLUEROV2_HEAVY, CONFIGS, vehicle_variant, initial_state,
                           action_frames, param_multipliers, env_classes)

    c = CONFIGS["c3"]
    E, T, S = args.n_envs, args.n_ctrl, c.substeps
    classes = [vehicle_variant(BLUEROV2, thr_map=1, thr_tau=0.05),
               vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)]
    cls = env_classes(E, "halves")
    n_b = int((cls == 0).sum())
    n_h = E - n_b
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # inputs, resident in HBM before timing
    x0 = torch.from_numpy(initial_state(E, 21, c.seed_base + 2)).to(dev)
    mult = torch.from_numpy(param_multipliers(E, c.rho, c.seed_base + 1)).to(dev)
    act = torch.empty((T, 8, E), dtype=torch.float32, device=dev)
    for t, fr in enumerate(action_frames(T, 8, E, c.seed_base + 3)):
        act[t].copy_(torch.from_numpy(fr))
    stats = torch.empty((T, 4), dtype=torch.float64, device=dev)

    sim = mg.Sim(classes, E, c.dt_sub, S, env_class=cls)

    def step(plain=False):
        sim.reset(state=x0, param_mult=mult)
        sim.rollout(act, stats=stats, plain=plain)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    env_substeps = E * T * S
    value = env_substeps * args.steps / wall

    # dominant kernel: the fused step, timed alone (graph replays only) with HIP events
    sim.reset(state=x0, param_mult=mult)
    sim.rollout(act, stats=stats)            # graph already cached
    torch.cuda.synchronize()
    reps = max(2, args.steps)
    ev0.record(stream)
    for _ in range(reps):
        sim.rollout(act, stats=stats)
    ev1.record(stream)
    torch.cuda.synchronize()
    fused_ms = ev0.elapsed_time(ev1) / reps
    flops_rollout = (n_b * substep_flops(6, True, S) + n_h * substep_flops(8, True, S)) * T * S
    executed = flops_rollout / (fused_ms * 1e-3)
    algo_flops_rollout = ALGO_FLOPS_PER_ENV_SUBSTEP * E * S * T
    achieved = algo_flops_rollout / (fused_ms * 1e-3)
    traffic = load_traffic("k_step_fused_control_step")
    algo_bytes_ctrl = n_b * fused_algo_bytes(6, True) + n_h * fused_algo_bytes(8, True)
    st = stats.cpu().numpy()

    out = {
        "metric": METRIC, "value": value, "unit": "env-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c3: 1,048,576 envs (half BlueROV2 / half BlueROV2 Heavy), "
                               "+-20% randomisation, quadratic thrust + 0.05 s lag, "
                               "200 control steps x 16 RK4 sub-steps of 5 ms per step, "
                               "fused launch per control step from a HIP graph",
                   "n_envs": E, "control_steps": T, "substeps_per_launch": S, "dt_sub": c.dt_sub},
        "env_control_steps_per_s": E * T * args.steps / wall,
        "sim_seconds_per_wall_second": value * c.dt_sub,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU,
                     "traffic": traffic,
                     "kernel": "k_step<6|8,lag> fused: the BlueROV2 and Heavy launches of one "
                               "control step (16 RK4 sub-steps each), run concurrently",
                     "control_step_us": fused_ms * 1e3 / T,
                     "counted": f"algorithmic: {ALGO_FLOPS_PER_ENV_SUBSTEP:.0f} flop per "
                                "env-substep (structured RK4 step) x env-substeps per launch",
                     "algorithmic_flops_per_control_step": algo_flops_rollout / T,
                     "executed": {"achieved": executed / 1e12,
                                  "frac": executed / PEAK_FP32_VALU,
                                  "flops_per_control_step": flops_rollout / T,
                                  "flops_per_env_substep": {
                                      "bluerov2": substep_flops(6, True, S),
                                      "heavy": substep_flops(8, True, S)},
                                  "counted": "the kernel's own formulation, instruction by "
                                             "instruction (SQ_INSTS_VALU_FLOPS_FP32 agrees)"},
                     "algorithmic_bytes_per_control_step": algo_bytes_ctrl,
                     "traffic_ratio": None if traffic is None else traffic / algo_bytes_ctrl},
        "stats_last_step": {"mean_dist": st[-1, 0] / max(1, E - st[-1, 3]),
                            "max_dist": st[-1, 1], "nonfinite": st[-1, 3]},
    }

    progress(f"fused rollout timed: {ms_step:.2f} ms per step")
    if not args.no_plain:
        sim.reset(state=x0, param_mult=mult)
        sim.rollout(act, stats=stats, plain=True)     # capture
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(2):
            sim.rollout(act, stats=stats, plain=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        plain_ms = ev0.elapsed_time(ev1) / 2
        bytes_rollout = (n_b * plain_bytes(6, True) + n_h * plain_bytes(8, True)) * T * S
        out["plain"] = {
            "env_steps_per_s": env_substeps / (plain_ms * 1e-3),
            "ms_per_rollout": plain_ms, "launches": 2 * T * S,
            "avg_launch_us": plain_ms * 1e3 / (2 * T * S),
            "achieved_GBps_algorithmic": bytes_rollout / (plain_ms * 1e-3) / 1e9,
            "frac_hbm": bytes_rollout / (plain_ms * 1e-3) / PEAK_HBM,
            "speedup_fused_vs_plain": plain_ms / fused_ms,
        }
        # the same 6400 launches issued one by one from the host (mg_step_plain, no graph)
        sim.reset(state=x0, param_mult=mult)
        torch.cuda.synchronize()
        ev0.record(stream)
        sim.step(act, stats=stats, plain=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        eager_ms = ev0.elapsed_time(ev1)
        out["plain"]["uncaptured"] = {
            "env_steps_per_s": env_substeps / (eager_ms * 1e-3), "ms_per_rollout": eager_ms,
            "avg_launch_us": eager_ms * 1e3 / (2 * T * S),
            "frac_hbm": bytes_rollout / (eager_ms * 1e-3) / PEAK_HBM}
        progress("plain comparator timed")
    if not args.no_task:
        out["task_epilogue"] = bench_task(torch, sim, act, x0, n_b, n_h)
        progress("task epilogue timed")
    if not args.no_split:
        out["split_scheme"] = bench_split(torch, mg, classes, cls, act, x0, mult)
        progress("split scheme timed")
    sim.close()
    del act
    torch.cuda.empty_cache()

    if not args.no_policy:
        out["policy_in_the_loop"] = [bench_policy(torch, mg, n) for n in (4096, 1 << 16, 1 << 20)]
        out["policy_in_the_loop"] += [bench_policy(torch, mg, n, graph=True)
                                      for n in (4096, 1 << 16)]
        progress("policy in the loop timed")
    if not args.no_adjoint:
        out["adjoint"] = bench_adjoint(torch, mg)
        out["adjoint_1m_envs"] = bench_adjoint(torch, mg, reps=3, n_envs=1 << 20)
        progress("adjoint timed")
    if not args.no_serve:
        cb = bench_serving(torch, mg, args.serve_seconds, warmup_s=args.serve_warmup,
                           steps_per_tick=8)
        progress(f"serving (continuous batching) timed: p99 {cb['p99_ms']:.3f} ms")
        cb1 = bench_serving(torch, mg, args.serve_aux_seconds, warmup_s=1.0, steps_per_tick=1)
        progress("serving (one step per tick) timed")
        base = bench_serving(torch, mg, args.serve_seconds, warmup_s=args.serve_warmup,
                             fifo_plain=True)
        progress(f"serving (FIFO baseline) timed: p99 {base['p99_ms']:.3f} ms")
        out["serving"] = {"continuous_batching": cb, "continuous_batching_1_step_per_tick": cb1,
                          "baseline_fifo_plain": base,
                          "p99_speedup_vs_baseline": base["p99_ms"] / cb["p99_ms"]}
    out["cpu_baseline"] = None if args.no_cpu else cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
