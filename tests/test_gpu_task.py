"""GPU parity of the Gym-style task step (mg_task_*, Sec. III) against the oracle.

The physics of a task step is exactly mg_step's (bitwise); the epilogue (error of
Eq. (4), episode end and automatic reset, observation of Eq. (2)) is compared with
the oracle's task rollout on the same inputs: done flags and counters exactly,
errors, observations and states within 1e-4 over 11 control steps (the one-step
tolerance 1e-5 accumulated), angles modulo 2 pi; and, from the GPU's own state, the
observation within 1e-6 (the epilogue is FP64 on both sides).
"""
import math

import numpy as np
import pytest

from workloads import (BLUEROV2, BLUEROV2_HEAVY, vehicle_variant, initial_state, actions,
                       param_multipliers, env_classes)
from tests.gpu_util import dev, host, rel_err, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CLASSES = [vehicle_variant(BLUEROV2, thr_map=1, thr_tau=0.05),
           vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)]
S, DT, D = 4, 0.005, 21
TOL_TASK = 1e-4


@pytest.fixture(scope="module")
def mgmod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_14117_amd import mg
    mg.lib()
    return mg


def _task(kind, **kw):
    t = {"task": kind, "lookahead": 4, "radius": 1.5, "omega": 0.4, "climb_rate": 0.05,
         "lookahead_dt": 0.0, "episode_steps": 1 << 30, "max_error": 0.0}
    t.update(kw)
    return t


def _inputs(E, T, seed):
    cls = env_classes(E, "bernoulli", seed) if seed % 2 else env_classes(E, "halves")
    x0 = initial_state(E, D, seed + 1)
    x0[19:, cls == 0] = 0
    act = actions(T, 8, E, seed + 2)
    mult = param_multipliers(E, 0.2, seed + 3)
    rng = np.random.default_rng(seed + 4)
    center = rng.normal(0, 0.3, (3, E)).astype(np.float32)
    phase = rng.uniform(0, 2 * math.pi, E).astype(np.float32)
    yaw = rng.uniform(-math.pi, math.pi, E).astype(np.float32)
    rs = initial_state(E, D, seed + 5)
    rs[19:, cls == 0] = 0
    rm = param_multipliers(E, 0.2, seed + 6)
    return cls, x0, act, mult, center, phase, yaw, rs, rm


def _angle_rows(obs_dim):
    m = (obs_dim - 6) // 6
    return [6 * i + r for i in range(m) for r in (3, 4, 5)]


def _obs_err(got, ref):
    """rel_err with the angle rows compared modulo 2 pi."""
    got = np.asarray(got, np.float64).copy()
    ref = np.asarray(ref, np.float64)
    rows = _angle_rows(got.shape[-2])
    d = got[..., rows, :] - ref[..., rows, :]
    got[..., rows, :] = ref[..., rows, :] + np.remainder(d + np.pi, 2 * np.pi) - np.pi
    return rel_err(got, ref)


def test_task_step_physics_equals_mg_step(mgmod):
    """Without episode ends a task step advances the state exactly as mg_step does."""
    E, T = 3000 + 37, 5
    cls, x0, act, mult, center, phase, yaw, _, _ = _inputs(E, T, 11)
    say("task physics vs mg_step")
    a = mgmod.Sim(CLASSES, E, DT, S, env_class=cls)
    b = mgmod.Sim(CLASSES, E, DT, S, env_class=cls)
    for s in (a, b):
        s.reset(state=dev(x0), param_mult=dev(mult))
    b.task_configure(_task("circle"), dev(center), dev(phase), dev(yaw))
    act_d = dev(act)
    for t in range(T):
        a.step(act_d[t:t + 1])
        b.task_step(act_d[t])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(a.get_state()), host(b.get_state()))
    assert np.all(host(b.task_counters()) == T)
    a.close()
    b.close()


def _oracle_run(oracle, tk, cls, x0, act, mult, center, phase, yaw, rs, rm):
    return oracle.task_rollout(CLASSES, tk, x0, act, S, DT, center, phase, yaw, env_class=cls,
                               mult=mult, reset_state=rs, reset_mult=rm)


def _bound_without_ties(oracle, kind, inputs):
    """An error bound that some envs cross and no oracle error lies within 2e-5 of (twenty
    times the FP32 path's error difference over these steps), so the flags cannot differ
    from the oracle's by rounding."""
    cls, x0, act, mult, center, phase, yaw, rs, rm = inputs
    free = _oracle_run(oracle, _task(kind, episode_steps=4), cls, x0, act, mult, center, phase,
                       yaw, rs, rm)
    emax = float(np.quantile(free["err"], 0.8))
    for _ in range(50):
        ref = _oracle_run(oracle, _task(kind, episode_steps=4, max_error=emax), cls, x0, act, mult,
                          center, phase, yaw, rs, rm)
        if np.min(np.abs(ref["err"] - emax)) > 2e-5:
            return emax, ref
        emax += 5.3e-5
    raise AssertionError("no tie-free error bound found")


@pytest.mark.parametrize("kind", ["station", "circle", "helix", "lemniscate"])
def test_task_rollout_matches_oracle(mgmod, oracle, kind):
    """11 Gym steps with episodes of 4 steps and an error bound: flags and counters exact,
    errors, observations (angles modulo 2 pi) and states within 1e-4 of the oracle."""
    E, T = 2000 + 37, 11
    inputs = _inputs(E, T, 20 + 10 * list(("station", "circle", "helix", "lemniscate")).index(kind))
    cls, x0, act, mult, center, phase, yaw, rs, rm = inputs
    emax, ref = _bound_without_ties(oracle, kind, inputs)
    assert (ref["done"] == 1).any() and (ref["done"] == 2).any()
    say(f"task {kind} rollout, E={E}, max_error={emax:.4f}")
    sim = mgmod.Sim(CLASSES, E, DT, S, env_class=cls)
    sim.reset(state=dev(x0), param_mult=dev(mult))
    sim.task_configure(_task(kind, episode_steps=4, max_error=emax), dev(center), dev(phase),
                       dev(yaw))
    obs0 = host(sim.task_observe())
    act_d, rs_d, rm_d = dev(act), dev(rs), dev(rm)
    obs, err, done = [obs0], [], []
    for t in range(T):
        o, e, d = sim.task_step(act_d[t], reset_state=rs_d, reset_mult=rm_d)
        obs.append(host(o).copy())
        err.append(host(e).copy())
        done.append(host(d).copy())
    xT, kT = host(sim.get_state()), host(sim.task_counters())
    sim.close()
    np.testing.assert_array_equal(np.array(done), ref["done"])
    np.testing.assert_array_equal(kT, ref["k"])
    assert rel_err(np.array(err), ref["err"]) <= TOL_TASK
    assert _obs_err(np.array(obs), ref["obs"]) <= TOL_TASK
    assert rel_err(xT, ref["x"]) <= TOL_TASK


def test_observation_from_the_gpu_state(mgmod, oracle):
    """The epilogue's observation equals the oracle's of the GPU's own FP32 state and
    counters to 1e-6 (FP64 on both sides)."""
    E, T = 1500 + 11, 3
    cls, x0, act, mult, center, phase, yaw, rs, rm = _inputs(E, T, 61)
    for kind in ("station", "circle", "helix", "lemniscate"):
        say(f"task {kind} local observation")
        tk = _task(kind, episode_steps=2, lookahead=6, lookahead_dt=0.05)
        sim = mgmod.Sim(CLASSES, E, DT, S, env_class=cls)
        sim.reset(state=dev(x0), param_mult=dev(mult))
        sim.task_configure(tk, dev(center), dev(phase), dev(yaw))
        act_d = dev(act)
        for t in range(T):
            o, _, _ = sim.task_step(act_d[t], reset_state=dev(rs))
        got = host(o)
        x, k = host(sim.get_state()), host(sim.task_counters())
        sim.close()
        ref = oracle.task_observe(tk, x, center, phase, yaw, k, S * DT)
        assert _obs_err(got, ref) <= 1e-6


def test_reset_zeroes_episode_counters(mgmod):
    E = 300
    cls, x0, act, mult, center, phase, yaw, _, _ = _inputs(E, 3, 71)
    say("task counters and mg_reset")
    sim = mgmod.Sim(CLASSES, E, DT, S, env_class=cls)
    sim.reset(state=dev(x0))
    sim.task_configure(_task("helix"), dev(center), dev(phase))
    act_d = dev(act)
    for t in range(3):
        sim.task_step(act_d[t])
    ids = torch.tensor([0, 7, 299], dtype=torch.int64, device="cuda")
    sim.reset(env_ids=ids, state=dev(x0[:, [0, 7, 299]]))
    k = host(sim.task_counters())
    sim.close()
    expect = np.full(E, 3, np.int32)
    expect[[0, 7, 299]] = 0
    np.testing.assert_array_equal(k, expect)


def test_nonfinite_env_terminates_and_restarts(mgmod):
    """A non-positive-definite mass matrix makes an env non-finite: its reset flags it
    MG_FLAG_NOT_SPD, the task step reports done 1 and restarts it from its reset state with
    the reset multipliers (finite again at the next step), which clears the flag."""
    E = 64
    cls, x0, act, mult, center, phase, yaw, rs, _ = _inputs(E, 2, 81)
    mult = mult.copy()
    mult[0, 5] = -50.0
    say("task non-finite env")
    sim = mgmod.Sim(CLASSES, E, DT, S, env_class=cls)
    sim.reset(state=dev(x0), param_mult=dev(mult))
    sim.task_configure(_task("station", episode_steps=100), dev(center), dev(phase), dev(yaw))
    act_d, rs_d = dev(act), dev(rs)
    fl = host(sim.get_flags())
    assert fl[5] == 2 and np.count_nonzero(fl) == 1
    ones = torch.ones((23, E), dtype=torch.float32, device="cuda")
    _, _, d0 = sim.task_step(act_d[0], reset_state=rs_d, reset_mult=ones)
    d0 = host(d0).copy()
    assert np.count_nonzero(host(sim.get_flags())) == 0
    o1, _, d1 = sim.task_step(act_d[1], reset_state=rs_d, reset_mult=ones)
    d1, o1 = host(d1), host(o1)
    sim.close()
    assert d0[5] == 1 and np.sum(d0 != 0) == 1
    assert np.all(d1 == 0) and np.all(np.isfinite(o1))


def test_task_step_captured_in_a_graph(mgmod):
    """mg_task_step captured in a HIP graph (through torch.cuda.graph, with the class
    launches forked onto the sim's helper streams inside the capture) and replayed three
    times, with eager work and synchronisations between the replays, matches an eager
    twin after every replay bitwise."""
    E = 4096 + 5
    cls, x0, act, mult, center, phase, yaw, rs, _ = _inputs(E, 4, 91)
    say("task step graph capture")
    tk = _task("lemniscate", episode_steps=2)
    sims = []
    for _ in range(2):
        s = mgmod.Sim(CLASSES, E, DT, S, env_class=cls)
        s.reset(state=dev(x0), param_mult=dev(mult))
        s.task_configure(tk, dev(center), dev(phase), dev(yaw))
        sims.append(s)
    eager, capt = sims
    a_d, rs_d = dev(act), dev(rs)
    a_static = a_d[0].clone()
    bufs = [torch.empty((eager.obs_dim, E), device="cuda"), torch.empty((E,), device="cuda"),
            torch.empty((E,), dtype=torch.int32, device="cuda")]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        capt.task_step(a_static, *bufs, reset_state=rs_d)
    torch.cuda.synchronize()
    for t in range(3):
        a_static.copy_(a_d[t])
        g.replay()
        o, e, d = eager.task_step(a_d[t], reset_state=rs_d)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(host(bufs[0]), host(o))
        np.testing.assert_array_equal(host(bufs[1]), host(e))
        np.testing.assert_array_equal(host(bufs[2]), host(d))
        np.testing.assert_array_equal(host(capt.get_state()), host(eager.get_state()))
        _ = torch.ones(1000, device="cuda").sum()     # eager work between replays
    eager.close()
    capt.close()


@pytest.mark.slow
def test_full_size_circle_task_sampled(mgmod, oracle):
    """The benchmark's task configuration: 2^20 envs (half BlueROV2, half Heavy), 16 sub-steps
    of 5 ms per control step, circle tracking with 4 look-ahead points, episodes of 100.
    After 3 task steps every counter is 3, no env is done, and the observation of 256 envs
    spread over both classes (and the last env) equals the oracle's of the GPU's own state."""
    E, S16, T = 1 << 20, 16, 3
    cls = env_classes(E, "halves")
    x0 = initial_state(E, D, 901)
    x0[19:, cls == 0] = 0
    g = torch.Generator(device="cuda").manual_seed(902)
    act = torch.rand((T, 8, E), generator=g, device="cuda") * 2 - 1
    phase = (np.random.default_rng(903).uniform(0, 2 * math.pi, E)).astype(np.float32)
    center = np.zeros((3, E), np.float32)
    tk = {"task": "circle", "lookahead": 4, "radius": 2.0, "omega": 0.5, "episode_steps": 100}
    say("task full size circle")
    sim = mgmod.Sim(CLASSES, E, DT, S16, env_class=cls)
    sim.reset(state=dev(x0))
    sim.task_configure(tk, dev(center), dev(phase))
    for t in range(T):
        obs, err, done = sim.task_step(act[t])
    torch.cuda.synchronize()
    k = host(sim.task_counters())
    assert np.all(k == T)
    assert int(done.abs().sum()) == 0 and bool(torch.isfinite(err).all())
    idx = np.unique(np.r_[np.linspace(0, E - 1, 256).astype(np.int64), E - 1])
    it = torch.from_numpy(idx).to("cuda")
    got = host(obs[:, it])
    x = host(sim.get_state()[:, it])
    sim.close()
    ref = oracle.task_observe(tk, x, center[:, idx], phase[idx], np.zeros(idx.size, np.float32),
                              k[idx], S16 * DT)
    assert _obs_err(got, ref) <= 1e-6
