"""GPU parity of the HIP step path (through the C ABI) against the FP64 oracle.

Tolerances: one control step <= 1e-5 and whole trajectories <= 1e-3 in the
norm max |x_gpu - x_ref| / max(1, |x_ref|), from identical FP32 inputs.
"""
import numpy as np
import pytest

from workloads import (BLUEROV2, BLUEROV2_HEAVY, CONFIGS, vehicle_variant, initial_state,
                       random_states, actions, action_frames, param_multipliers, env_classes)
from tests.gpu_util import dev, host, rel_err, say, TOL_ONE_STEP, TOL_TRAJ

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mgmod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_14117_amd import mg
    mg.lib()
    return mg


LAGGED = {
    "bluerov2": vehicle_variant(BLUEROV2, thr_map=1, thr_tau=0.05),
    "heavy": vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05),
}


def _run(mgmod, classes, x0, act, dt, S, env_class=None, mult=None, targets=None, mode="fused"):
    E = x0.shape[1]
    sim = mgmod.Sim(classes, E, dt, S, env_class=env_class)
    sim.reset(state=dev(x0), param_mult=None if mult is None else dev(mult))
    T = act.shape[0]
    traj = torch.empty((T, sim.state_dim, E), dtype=torch.float32, device="cuda")
    stats = torch.empty((T, 4), dtype=torch.float64, device="cuda")
    a = dev(act)
    tg = None if targets is None else dev(targets)
    if mode == "fused":
        sim.step(a, targets=tg, traj=traj, stats=stats)
    elif mode == "plain":
        sim.step(a, targets=tg, traj=traj, stats=stats, plain=True)
    else:
        sim.rollout(a, targets=tg, traj=traj, stats=stats, plain=(mode == "graph_plain"))
    torch.cuda.synchronize()
    out = host(traj), host(stats), host(sim.get_state())
    sim.close()
    return out


def test_c1_full_trajectory(mgmod, oracle):
    c = CONFIGS["c1"]
    say("c1 64 envs x 1000 steps, fused single launch")
    x0 = initial_state(c.n_envs, 13, c.seed_base + 2)
    act = actions(c.n_ctrl, 6, c.n_envs, c.seed_base + 3)
    traj, stats, xT = _run(mgmod, BLUEROV2, x0, act, c.dt_sub, c.substeps)
    ref = oracle.rollout(BLUEROV2, x0, act, c.substeps, c.dt_sub, want_traj=True, want_stats=True)
    assert rel_err(traj[0], ref["traj"][0]) <= TOL_ONE_STEP
    assert rel_err(traj, ref["traj"]) <= TOL_TRAJ
    np.testing.assert_array_equal(xT, traj[-1])
    assert np.all(stats[:, 3] == 0)
    np.testing.assert_allclose(stats[:, :3], ref["stats"][:, :3], rtol=1e-4)


@pytest.mark.parametrize("variant", ["c1_linear", "c2_heavy_lag", "mixed_lag"])
def test_one_control_step_over_the_envelope(mgmod, oracle, variant):
    """One control step from states spread over the operating envelope (random attitude,
    up to 1.5 m/s and 2 rad/s, saturated thrusters), ragged env count, randomised params."""
    E = 4096 + 37
    if variant == "c1_linear":
        classes, cls, dt, S, D, N = [BLUEROV2], None, 0.01, 1, 13, 6
    elif variant == "c2_heavy_lag":
        classes, cls, dt, S, D, N = [LAGGED["heavy"]], None, 0.005, 4, 21, 8
    else:
        classes, dt, S, D, N = [LAGGED["bluerov2"], LAGGED["heavy"]], 0.005, 4, 21, 8
        cls = env_classes(E, "bernoulli", 99)
    say("one step", variant, E)
    x0 = random_states(E, D, 31)
    if cls is not None:
        x0[19:, cls == 0] = 0.0
    act = actions(1, N, E, 32) * np.float32(1.3)      # some throttles saturate
    mult = param_multipliers(E, 0.2, 33)
    traj, stats, _ = _run(mgmod, classes, x0, act, dt, S, env_class=cls, mult=mult)
    ref = oracle.rollout(classes, x0, act, S, dt, env_class=cls, mult=mult, want_traj=True,
                         want_stats=True)
    assert rel_err(traj[0], ref["traj"][0]) <= TOL_ONE_STEP
    np.testing.assert_allclose(stats[0, :3], ref["stats"][0, :3], rtol=1e-5)
    assert stats[0, 3] == ref["stats"][0, 3] == 0


def test_c2_trajectory_on_env_subset(mgmod, oracle):
    c = CONFIGS["c2"]
    v = LAGGED["heavy"]
    say("c2 4096 heavy x 1000 control x 4 substeps, graph rollout")
    x0 = initial_state(c.n_envs, 21, c.seed_base + 2)
    act = actions(c.n_ctrl, 8, c.n_envs, c.seed_base + 3)
    mult = param_multipliers(c.n_envs, c.rho, c.seed_base + 1)
    traj, stats, xT = _run(mgmod, v, x0, act, c.dt_sub, c.substeps, mult=mult, mode="graph")
    sub = np.arange(0, c.n_envs, 8)
    ref = oracle.rollout(v, x0[:, sub], act[:, :, sub], c.substeps, c.dt_sub, mult=mult[:, sub],
                         want_traj=True)
    assert rel_err(traj[0][:, sub], ref["traj"][0]) <= TOL_ONE_STEP
    assert rel_err(traj[:, :, sub], ref["traj"]) <= TOL_TRAJ
    # full-env statistics against the oracle's, over all 4096 envs for the last step only
    full = oracle.rollout(v, x0, act[:2], c.substeps, c.dt_sub, mult=mult, want_stats=True)
    _, st2, _ = _run(mgmod, v, x0, act[:2], c.dt_sub, c.substeps, mult=mult)
    np.testing.assert_allclose(st2[:, :3], full["stats"][:, :3], rtol=1e-5)


def test_fused_plain_graph_agree(mgmod):
    """One fused launch of n_ctrl x S sub-steps and per-control-step graph launches give the
    same states and statistics bitwise; the plain per-sub-step kernel (eager or graph) agrees
    bitwise with itself and with the fused kernel to rounding (it re-forms the lag wrench from
    the stored thrust every sub-step instead of carrying it)."""
    E, T = 3000, 40
    classes = [LAGGED["bluerov2"], LAGGED["heavy"]]
    cls = env_classes(E, "halves")
    x0 = initial_state(E, 21, 41)
    x0[19:, cls == 0] = 0
    act = actions(T, 8, E, 42)
    mult = param_multipliers(E, 0.2, 43)
    tgt = np.random.default_rng(44).normal(size=(3, E)).astype(np.float32)
    res = {}
    for mode in ["fused", "plain", "graph", "graph_plain"]:
        say("mode", mode)
        res[mode] = _run(mgmod, classes, x0, act, 0.005, 4, env_class=cls, mult=mult,
                         targets=tgt, mode=mode)
    np.testing.assert_array_equal(res["graph"][0], res["fused"][0])
    np.testing.assert_array_equal(res["graph"][1], res["fused"][1])
    np.testing.assert_array_equal(res["graph_plain"][0], res["plain"][0])
    np.testing.assert_array_equal(res["graph_plain"][1], res["plain"][1])
    assert rel_err(res["plain"][0], res["fused"][0]) <= 1e-5
    np.testing.assert_allclose(res["plain"][1], res["fused"][1], rtol=1e-5)


def test_interleaved_classes_match_contiguous(mgmod, oracle):
    """Envs of two classes in arbitrary order are regrouped internally; results come back in
    the caller's order and equal a contiguous layout bitwise."""
    E, T = 1000, 25
    classes = [LAGGED["bluerov2"], LAGGED["heavy"]]
    cls = env_classes(E, "bernoulli", 51)
    order = np.argsort(cls, kind="stable")
    x0 = initial_state(E, 21, 52)
    x0[19:, cls == 0] = 0
    act = actions(T, 8, E, 53)
    mult = param_multipliers(E, 0.2, 54)
    say("interleaved classes", E)
    tr_i, st_i, _ = _run(mgmod, classes, x0, act, 0.005, 4, env_class=cls, mult=mult)
    tr_c, st_c, _ = _run(mgmod, classes, x0[:, order], act[:, :, order], 0.005, 4,
                         env_class=cls[order], mult=mult[:, order])
    np.testing.assert_array_equal(tr_i[:, :, order], tr_c)
    np.testing.assert_allclose(st_i, st_c, rtol=1e-12)
    ref = oracle.rollout(classes, x0, act, 4, 0.005, env_class=cls, mult=mult, want_traj=True)
    assert rel_err(tr_i, ref["traj"]) <= 1e-4


@pytest.mark.parametrize("E", [1, 63, 65, 257, 1000])
def test_ragged_sizes(mgmod, oracle, E):
    say("ragged", E)
    v = LAGGED["heavy"]
    x0 = initial_state(E, 21, 61)
    act = actions(50, 8, E, 62)
    mult = param_multipliers(E, 0.2, 63)
    tr, st, _ = _run(mgmod, v, x0, act, 0.005, 4, mult=mult)
    ref = oracle.rollout(v, x0, act, 4, 0.005, mult=mult, want_traj=True, want_stats=True)
    assert rel_err(tr[0], ref["traj"][0]) <= TOL_ONE_STEP
    assert rel_err(tr, ref["traj"]) <= 1e-4
    np.testing.assert_allclose(st[:, :3], ref["stats"][:, :3], rtol=1e-5)


def test_reset_subset_params_and_resume(mgmod):
    E = 300
    v = LAGGED["heavy"]
    sim = mgmod.Sim(v, E, 0.005, 4)
    mult = param_multipliers(E, 0.2, 71)
    x0 = initial_state(E, 21, 72)
    sim.reset(state=dev(x0), param_mult=dev(mult))
    # absolute parameters are nominal x multiplier, rounded once to FP32
    nominal = np.array([v["mass"], *v["inertia"], *v["added_mass"], *v["d_lin"], *v["d_quad"],
                        v["buoyancy"]])
    expect = (nominal[:, None] * mult.astype(np.float64)).astype(np.float32)
    np.testing.assert_array_equal(host(sim.get_params()), expect)
    np.testing.assert_array_equal(host(sim.get_state()), x0)
    # partial reset of three envs
    ids = torch.tensor([5, 17, 299], dtype=torch.int64, device="cuda")
    xs = random_states(3, 21, 73)
    sim.reset(env_ids=ids, state=dev(xs), param_mult=dev(np.ones((23, 3), np.float32)))
    got = host(sim.get_state())
    expect_x = x0.copy()
    expect_x[:, [5, 17, 299]] = xs
    np.testing.assert_array_equal(got, expect_x)
    p = host(sim.get_params())
    np.testing.assert_array_equal(p[:, 17], nominal.astype(np.float32))
    np.testing.assert_array_equal(p[:, 16], expect[:, 16])
    # checkpoint / resume is bitwise
    act = dev(actions(20, 8, E, 74))
    sim.step(act[:10])
    snap_x = sim.get_state().clone()
    snap_p = sim.get_params().clone()
    sim.step(act[10:])
    ref = host(sim.get_state())
    sim2 = mgmod.Sim(v, E, 0.005, 4)
    sim2.set_params(snap_p)
    sim2.set_state(snap_x)
    sim2.step(act[10:])
    np.testing.assert_array_equal(host(sim2.get_state()), ref)
    sim.close()
    sim2.close()


@pytest.mark.parametrize("mode", ["fused", "graph"])
def test_nonfinite_env_is_frozen_flagged_and_counted(mgmod, mode):
    """Env 200's mass multiplier is -2 (M not positive definite): mg_reset flags it
    MG_FLAG_NOT_SPD and it is never stepped: its initial state throughout.  Env 100 gets a
    NaN throttle at control step 3: its state goes non-finite there and, at the end of that
    launch, goes back to the launch's input and is flagged MG_FLAG_NONFINITE -- with the 12
    control steps in one launch (fused) to x0, with one launch per control step (graph
    rollout) to its last finite state, which later launches keep.  Every other env equals,
    bitwise, the same run without the NaN; the statistics count the frozen and non-finite
    envs; mg_set_state clears the non-finite flag and a reset with valid multipliers clears
    the other."""
    E, T = 512, 12
    v = LAGGED["heavy"]
    x0 = initial_state(E, 21, 81)
    act = actions(T, 8, E, 82)
    bad = act.copy()
    bad[3, 1, 100] = np.nan
    mult = param_multipliers(E, 0.2, 83)
    mult[0, 200] = -2.0                  # mass -23 kg: M not positive definite

    def run(a):
        sim = mgmod.Sim(v, E, 0.005, 4)
        sim.reset(state=dev(x0), param_mult=dev(mult))
        traj = torch.empty((T, 21, E), dtype=torch.float32, device="cuda")
        stats = torch.empty((T, 4), dtype=torch.float64, device="cuda")
        if mode == "fused":
            sim.step(dev(a), traj=traj, stats=stats)
        else:
            sim.rollout(dev(a), traj=traj, stats=stats)
        return sim, host(traj), host(stats), host(sim.get_flags())

    say(f"non-finite, {mode}")
    sim_ok, tr_ok, st_ok, fl_ok = run(act)
    sim_bad, tr_bad, st_bad, fl_bad = run(bad)
    assert fl_ok[200] == 2 and fl_bad[200] == 2 and fl_bad[100] == 1
    assert np.count_nonzero(fl_ok) == 1 and np.count_nonzero(fl_bad) == 2
    for t in range(T):
        np.testing.assert_array_equal(tr_ok[t, :, 200], x0[:, 200])
    np.testing.assert_array_equal(tr_bad[:3, :, 100], tr_ok[:3, :, 100])
    assert not np.isfinite(tr_bad[3, :, 100]).all()
    if mode == "fused":
        np.testing.assert_array_equal(host(sim_bad.get_state())[:, 100], x0[:, 100])
    else:
        for t in range(4, T):
            np.testing.assert_array_equal(tr_bad[t, :, 100], tr_bad[2, :, 100])
        np.testing.assert_array_equal(host(sim_bad.get_state())[:, 100], tr_bad[2, :, 100])
    assert np.all(st_ok[:, 3] == 1)
    assert list(st_bad[:, 3]) == [1, 1, 1] + [2] * (T - 3)
    keep = np.setdiff1d(np.arange(E), [100])
    np.testing.assert_array_equal(tr_bad[:, :, keep], tr_ok[:, :, keep])
    # a new state clears the non-finite flag, valid multipliers the other
    sim_bad.set_state(dev(x0))
    assert list(np.flatnonzero(host(sim_bad.get_flags()))) == [200]
    sim_bad.reset(state=dev(x0), param_mult=dev(param_multipliers(E, 0.2, 83)))
    assert np.count_nonzero(host(sim_bad.get_flags())) == 0
    sim_ok.close()
    sim_bad.close()


def test_heave_steady_state_on_gpu(mgmod):
    """Closed form: d_l w + d_q w|w| = F for a pure heave thrust (no oracle involved)."""
    import math
    E, T = 64, 3000
    x0 = np.zeros((13, E), np.float32)
    x0[3] = 1
    act = np.zeros((T, 6, E), np.float32)
    act[:, 4:] = 0.5
    tr, _, _ = _run(mgmod, BLUEROV2, x0, act, 0.01, 1)
    F = -40.0
    w = -(-5.0 + math.sqrt(25 + 4 * 37 * 40.0)) / (2 * 37)
    np.testing.assert_allclose(tr[-1, 9], w, rtol=2e-6)
    assert np.abs(tr[-1, [7, 8, 10, 11, 12]]).max() < 1e-6
    assert np.abs(F) > 0


def test_run_to_run_determinism(mgmod):
    E, T = 20000, 30
    classes = [LAGGED["bluerov2"], LAGGED["heavy"]]
    cls = env_classes(E, "halves")
    x0 = initial_state(E, 21, 91)
    x0[19:, cls == 0] = 0
    act = actions(T, 8, E, 92)
    mult = param_multipliers(E, 0.2, 93)
    a = _run(mgmod, classes, x0, act, 0.005, 4, env_class=cls, mult=mult)
    b = _run(mgmod, classes, x0, act, 0.005, 4, env_class=cls, mult=mult)
    for u, w in zip(a, b):
        np.testing.assert_array_equal(u, w)


def test_graph_replays_match_eager(mgmod):
    """A captured rollout replayed several times, with eager work and synchronisation in
    between, reproduces the eager result on every replay."""
    E, T = 4096, 8
    v = LAGGED["heavy"]
    x0 = dev(initial_state(E, 21, 101))
    a = dev(actions(T, 8, E, 102))
    sim = mgmod.Sim(v, E, 0.005, 4)
    traj = torch.empty((T, 21, E), device="cuda")
    stats = torch.empty((T, 4), dtype=torch.float64, device="cuda")
    sim.reset(state=x0)
    sim.step(a, traj=traj, stats=stats)
    ref_traj, ref_stats = traj.clone(), stats.clone()
    for rep in range(3):
        say("replay", rep)
        traj.zero_()
        stats.zero_()
        sim.reset(state=x0)
        sim.rollout(a, traj=traj, stats=stats)
        torch.cuda.synchronize()
        assert torch.equal(traj, ref_traj) and torch.equal(stats, ref_stats)
        sim.reset(state=x0)
        sim.step(a[:3])                  # eager work between replays
        torch.cuda.synchronize()
    sim.close()


def _env_err(x_gpu, x_ref):
    """Per-env error in the norm of rel_err: max over components of |x - x_ref| / max(1, |x_ref|)."""
    x_gpu = np.asarray(x_gpu, np.float64)
    x_ref = np.asarray(x_ref, np.float64)
    return np.max(np.abs(x_gpu - x_ref) / np.maximum(1.0, np.abs(x_ref)), axis=0)


def _local_errors(oracle, classes, path, act, S, dt, cls, mult):
    """Local parity along a path: path [T+1][D][n] holds x0 and the states after each
    control step; the oracle advances every stored state by one control step (all T of them
    in one batch) and the result is compared with the next stored state.  Returns the
    per-env maximum over the T steps."""
    T1, D, n = path.shape
    T = T1 - 1
    starts = np.ascontiguousarray(path[:T].transpose(1, 0, 2).reshape(D, T * n))
    a = np.ascontiguousarray(act.transpose(1, 0, 2).reshape(1, act.shape[1], T * n))
    ref = oracle.rollout(classes, starts, a, S, dt, env_class=np.tile(cls, T),
                         mult=np.tile(mult, (1, T)))["x"]
    nxt = path[1:].transpose(1, 0, 2).reshape(D, T * n)
    return _env_err(nxt, ref).reshape(T, n).max(axis=0)


def _oracle_spread(oracle, classes, x0, act, S, dt, cls, mult, members=3, eta=1e-6, seed=7):
    """Conditioning of each env's trajectory: the FP64 oracle is run once clean and `members`
    times with a random perturbation of relative size eta (about ten times the FP32 path's
    typical one-step error) added to the state after every control step.  Returns the clean
    final state and, per env, the largest final deviation of a perturbed run from the clean
    one: how far local errors of that size carry the end state."""
    D, n = x0.shape
    rng = np.random.default_rng(seed)
    x = np.tile(np.asarray(x0, np.float64), (1, members + 1))
    ec, mm = np.tile(cls, members + 1), np.tile(mult, (1, members + 1))
    for t in range(act.shape[0]):
        x = oracle.rollout(classes, x, np.tile(act[t:t + 1], (1, 1, members + 1)), S, dt,
                           env_class=ec, mult=mm)["x"]
        noise = eta * rng.standard_normal((D, members * n)) * np.maximum(1.0, np.abs(x[:, n:]))
        x[:, n:] += noise
    clean = x[:, :n]
    spread = np.max([_env_err(x[:, (k + 1) * n:(k + 2) * n], clean) for k in range(members)],
                    axis=0)
    return clean, spread


@pytest.mark.slow
def test_c3_full_size_sampled(mgmod, oracle):
    """2^20 mixed envs, 16 sub-steps per launch, 200 launches from a graph, fused and plain.

    Every env stays finite with a unit quaternion.  On a sample (every 1024th env plus the
    envs where fused and plain end furthest apart) both paths are checked locally: each of
    the 200 control steps, restarted in the oracle from the path's own state, agrees to the
    one-step tolerance.  Over the whole horizon a few Heavy envs per 10^4 are ill-conditioned
    (random throttles drive them through the inverted attitude, where the CG-below-CB
    restoring moment is unstable): there the FP64 oracle itself moves by more than 1e-3 under
    perturbations of the size of FP32 rounding, so no FP32 path can match it to 1e-3.  The
    trajectory tolerance is asserted on the sampled envs whose oracle trajectory is
    well-conditioned (random perturbations of 1e-6 after every control step move the end state
    by at most the trajectory tolerance), which must be nearly all of them; on this workload
    the ill-conditioned envs move by 0.07 to 0.8 under those perturbations, the
    well-conditioned ones by 7e-5 at the median."""
    c = CONFIGS["c3"]
    E, T, S = c.n_envs, c.n_ctrl, c.substeps
    classes = [LAGGED["bluerov2"], LAGGED["heavy"]]
    cls = env_classes(E, "halves")
    x0 = initial_state(E, 21, c.seed_base + 2)
    x0[19:, cls == 0] = 0
    mult = param_multipliers(E, c.rho, c.seed_base + 1)
    say("c3 generate actions")
    frames = list(action_frames(T, 8, E, c.seed_base + 3))
    act = torch.empty((T, 8, E), dtype=torch.float32, device="cuda")
    for t, fr in enumerate(frames):
        act[t].copy_(torch.from_numpy(fr))
    sim = mgmod.Sim(classes, E, c.dt_sub, S, env_class=cls)
    final, trajs = {}, {}
    stats = torch.empty((T, 4), dtype=torch.float64, device="cuda")
    for mode in ("fused", "plain"):
        say(f"c3 {mode} graph rollout with trajectory")
        traj = torch.empty((T, 21, E), dtype=torch.float32, device="cuda")
        sim.reset(state=dev(x0), param_mult=dev(mult))
        sim.rollout(act, traj=traj, stats=stats if mode == "fused" else None,
                    plain=(mode == "plain"))
        final[mode] = host(sim.get_state())
        trajs[mode] = traj
    st = host(stats)
    sim.close()
    del act
    xf, xp = final["fused"], final["plain"]
    assert np.isfinite(xf).all() and np.isfinite(xp).all() and np.all(st[:, 3] == 0)
    np.testing.assert_allclose(np.linalg.norm(xf[3:7], axis=0), 1.0, atol=1e-6)
    np.testing.assert_array_equal(host(trajs["fused"][-1]), xf)

    d = _env_err(xp, xf)
    regular = np.arange(0, E, 1024)
    worst = np.argsort(-d)[:8]
    sample = np.unique(np.concatenate([regular, [0, E // 2 - 1, E // 2, E - 1], worst]))
    say(f"c3 fused vs plain at the end: max {d.max():.2e}, envs above 1e-3: {(d > 1e-3).sum()}")
    idx = torch.from_numpy(sample).cuda()
    act_s = np.stack([fr[:, sample] for fr in frames])
    cs, ms = cls[sample], mult[:, sample]
    for mode in ("fused", "plain"):
        path = np.concatenate([x0[None, :, sample],
                               host(trajs[mode].index_select(2, idx))], axis=0)
        trajs[mode] = None
        loc = _local_errors(oracle, classes, path, act_s, S, c.dt_sub, cs, ms)
        say(f"c3 {mode}: worst local one-step error {loc.max():.2e}")
        assert loc.max() <= TOL_ONE_STEP
    say("c3 oracle conditioning on the sample")
    clean, spread = _oracle_spread(oracle, classes, x0[:, sample], act_s, S, c.dt_sub, cs, ms)
    well = spread <= TOL_TRAJ
    in_regular = np.isin(sample, regular)
    say(f"c3 well-conditioned: {well[in_regular].sum()} of {in_regular.sum()} regular samples, "
        f"{well[np.isin(sample, worst)].sum()} of {len(worst)} most divergent envs")
    assert well[in_regular].mean() >= 0.98
    for x in (xf, xp):
        assert _env_err(x[:, sample[well]], clean[:, well]).max() <= TOL_TRAJ


def test_rollout_graph_cache_is_bounded(mgmod):
    """70 rollouts into 70 different trajectory buffers (more than the 64 cached graphs):
    every replay still writes the same, correct trajectory."""
    E, T = 64, 2
    x0 = initial_state(E, 13, 91)
    act = dev(actions(T, 6, E, 92))
    sim = mgmod.Sim(BLUEROV2, E, 0.01, 1)
    say("rollout graph cache bound")
    big = torch.zeros((70, T, 13, E), dtype=torch.float32, device="cuda")
    for i in range(70):
        sim.reset(state=dev(x0))
        sim.rollout(act, traj=big[i])
    torch.cuda.synchronize()
    ref = host(big[0])
    for i in range(1, 70):
        np.testing.assert_array_equal(host(big[i]), ref)
    sim.close()


@pytest.mark.parametrize("n_thr", [1, 3])
def test_few_thruster_classes(mgmod, oracle, n_thr):
    """Vehicles with 1 and 3 lagged thrusters (the smallest template instantiations),
    quadratic map, mixed with a BlueROV2 class: one control step and 30 steps vs the
    oracle."""
    E = 700
    small = vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)
    small = dict(small)
    small["thr_pos"] = small["thr_pos"][:n_thr]
    small["thr_dir"] = small["thr_dir"][:n_thr]
    classes = [LAGGED["bluerov2"], small]
    cls = env_classes(E, "bernoulli", 71)
    x0 = initial_state(E, 19, 72)
    x0[13 + n_thr:, cls == 1] = 0
    act = actions(30, 6, E, 73)
    mult = param_multipliers(E, 0.2, 74)
    say("few thrusters", n_thr)
    tr, _, _ = _run(mgmod, classes, x0, act, 0.005, 4, env_class=cls, mult=mult)
    ref = oracle.rollout(classes, x0, act, 4, 0.005, env_class=cls, mult=mult, want_traj=True)
    assert rel_err(tr[0], ref["traj"][0]) <= TOL_ONE_STEP
    assert rel_err(tr, ref["traj"]) <= 1e-4


@pytest.mark.parametrize("empty_first", [True, False])
def test_declared_class_without_envs(mgmod, empty_first):
    """A sim that declares a class no env belongs to (a lagged Heavy: its segment is empty,
    so every launcher skips it, while the I/O widths follow it: D = 21, N_max = 8) steps
    fused, per sub-step and from a graph, runs the split scheme and the adjoint exactly as
    a sim of the one populated class (BlueROV2, D = 13): bitwise, with the extra state and
    action rows zero.  The empty class comes first or second."""
    E, S, dt, T, K = 500, 4, 0.005, 6, 2
    heavy = LAGGED["heavy"]
    classes = [heavy, BLUEROV2] if empty_first else [BLUEROV2, heavy]
    cls = np.full(E, 1 if empty_first else 0, np.int32)
    x0 = initial_state(E, 13, 71)
    mult = param_multipliers(E, 0.2, 72)
    act6 = actions(T, 6, E, 73)
    g13 = np.random.default_rng(74).standard_normal((T, 13, E)).astype(np.float32)
    x0w, act8, g21 = (np.zeros((21, E), np.float32), np.zeros((T, 8, E), np.float32),
                      np.zeros((T, 21, E), np.float32))
    x0w[:13], act8[:, :6], g21[:, :13] = x0, act6, g13
    say("declared class without envs", "first" if empty_first else "second")
    res = {}
    for name, sim, xs, ac, g in (("one", mgmod.Sim(BLUEROV2, E, dt, S), x0, act6, g13),
                                 ("two", mgmod.Sim(classes, E, dt, S, env_class=cls), x0w,
                                  act8, g21)):
        D = sim.state_dim
        a = dev(ac)
        sim.reset(state=dev(xs), param_mult=dev(mult))
        traj = torch.empty((3, D, E), device="cuda")
        stats = torch.empty((3, 4), dtype=torch.float64, device="cuda")
        sim.step(a[:3], traj=traj, stats=stats)
        sim.step(a[3:4], plain=True)
        sim.rollout(a[4:6])
        r = {"traj": host(traj), "stats": host(stats), "state": host(sim.get_state())}
        sim.reset(state=dev(xs), param_mult=dev(mult))
        sim.step_split(a[:2])
        r["split"] = host(sim.get_state())
        sim.reset(state=dev(xs), param_mult=dev(mult))
        tr = torch.empty((T, D, E), device="cuda")
        ck, _ = sim.adj_forward(a, K, traj=tr)
        ga, gt, gx = sim.adj_backward(ck, a, K, dev(g))
        r.update(adj_traj=host(tr), gact=host(ga), gtheta=host(gt), gx0=host(gx))
        sim.close()
        res[name] = r
    one, two = res["one"], res["two"]
    np.testing.assert_array_equal(two["stats"], one["stats"])
    np.testing.assert_array_equal(two["gtheta"], one["gtheta"])
    for k in ("traj", "state", "split", "adj_traj", "gx0"):
        np.testing.assert_array_equal(two[k][..., :13, :], one[k], err_msg=k)
        assert (two[k][..., 13:, :] == 0).all(), k
    np.testing.assert_array_equal(two["gact"][:, :6], one["gact"])
    assert (two["gact"][:, 6:] == 0).all()


def test_invalid_calls_raise_and_leave_the_sim_usable(mgmod):
    """Zero control steps, a task step before a task is configured and a split step of zero
    control steps are rejected (MG_ERR_INVALID) without touching the state."""
    E = 64
    sim = mgmod.Sim(BLUEROV2, E, 0.01, 1)
    x0 = initial_state(E, 13, 81)
    sim.reset(state=dev(x0))
    act = dev(actions(1, 6, E, 82))
    say("invalid calls")
    with pytest.raises(mgmod.MgError):
        sim.step(act[:0])
    with pytest.raises(mgmod.MgError):
        sim.step_split(act[:0])
    with pytest.raises(mgmod.MgError):
        sim.obs_dim = 12
        sim.task_step(act[0])
    np.testing.assert_array_equal(host(sim.get_state()), x0)
    sim.step(act)
    assert np.isfinite(host(sim.get_state())).all()
    sim.close()


@pytest.mark.slow
def test_largest_env_count_offsets_beyond_32_bits(mgmod, oracle):
    """2^28 + 37 mixed envs with Bernoulli classes (the class permutation spans the whole
    range): state offsets reach 5.6e9 elements (22.5 GB), past any 32-bit index.  One
    control step of 2 sub-steps from device-generated inputs; every env stays finite, and
    128 envs spread over the range and at its end match the oracle within the one-step
    tolerance."""
    free = torch.cuda.mem_get_info()[0]
    if free < (230 << 30):
        pytest.skip(f"needs ~230 GB of free device memory, {free >> 30} GB free")
    E, S, dt = (1 << 28) + 37, 2, 0.005
    classes = [LAGGED["bluerov2"], LAGGED["heavy"]]
    cls = (np.random.default_rng(71).random(E) < 0.5).astype(np.int32)
    say(f"largest env count E={E}")
    g = torch.Generator(device="cuda").manual_seed(72)
    x0 = torch.empty((21, E), dtype=torch.float32, device="cuda")
    x0[0:3].uniform_(-1.0, 1.0, generator=g)
    x0[3:7].normal_(generator=g)
    x0[3:7] /= x0[3:7].norm(dim=0, keepdim=True)
    x0[7:13].uniform_(-0.5, 0.5, generator=g)
    x0[13:].uniform_(-20.0, 20.0, generator=g)
    act = torch.empty((1, 8, E), dtype=torch.float32, device="cuda").uniform_(-1.2, 1.2,
                                                                             generator=g)
    mult = torch.empty((23, E), dtype=torch.float32, device="cuda").uniform_(0.8, 1.2,
                                                                            generator=g)
    sim = mgmod.Sim(classes, E, dt, S, env_class=cls)
    sim.reset(state=x0, param_mult=mult)
    sim.step(act)
    out = sim.get_state()
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
    rng = np.random.default_rng(73)
    idx = np.unique(np.r_[0:32, E // 2 - 16:E // 2 + 16, E - 32:E,
                          rng.integers(0, E, 32)])
    it = torch.from_numpy(idx).to("cuda")
    xs, acts, ms = host(x0[:, it]), host(act[:, :, it]), host(mult[:, it])
    got = host(out[:, it])
    del out, x0, act, mult
    sim.close()
    torch.cuda.empty_cache()
    c = cls[idx]
    xs[19:, c == 0] = 0.0
    got[19:, c == 0] = 0.0
    ref = oracle.rollout(classes, xs, acts, S, dt, env_class=c, mult=ms)
    assert rel_err(got, ref["x"]) <= TOL_ONE_STEP


@pytest.mark.parametrize("n_thr,lag", [(2, False), (5, False), (7, True), (8, False)])
def test_other_instantiations(mgmod, oracle, n_thr, lag):
    """Thruster counts and lag settings the other step tests leave out (each is its own
    compiled kernel): 300 envs, one control step and 20 steps of 4 sub-steps vs the oracle."""
    v = dict(vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05 if lag else 0.0))
    v["thr_pos"] = v["thr_pos"][:n_thr]
    v["thr_dir"] = v["thr_dir"][:n_thr]
    D = 13 + (n_thr if lag else 0)
    E = 300
    x0 = random_states(E, D, 81)
    act = actions(20, n_thr, E, 82) * np.float32(1.2)
    mult = param_multipliers(E, 0.2, 83)
    say("step instantiation", n_thr, lag)
    tr, st, _ = _run(mgmod, v, x0, act, 0.005, 4, mult=mult)
    ref = oracle.rollout(v, x0, act, 4, 0.005, mult=mult, want_traj=True)
    assert rel_err(tr[0], ref["traj"][0]) <= TOL_ONE_STEP
    assert rel_err(tr, ref["traj"]) <= 1e-4
