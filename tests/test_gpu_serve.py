"""GPU tests of the continuous-batching serving loop (mg_server_*).

A request's final states must be the same (bitwise) alone, in a mix of
concurrently served requests and through mg_step, equal to rounding in the
FIFO baseline (plain per-sub-step kernel), and within the trajectory
tolerance of the FP64 oracle.
"""
import threading
import time

import numpy as np
import pytest

from workloads import (BLUEROV2, BLUEROV2_HEAVY, vehicle_variant, initial_state, actions,
                       param_multipliers, env_classes)
from workloads.gen import splitmix64_throttles
from tests.gpu_util import dev, host, rel_err, say, TOL_TRAJ

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CLASSES = [vehicle_variant(BLUEROV2, thr_map=1, thr_tau=0.05),
           vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)]
DT, S, D, NMAX = 0.005, 4, 21, 8
POOL = 40000     # columns of the shared device input pools
LMAX = 64


@pytest.fixture(scope="module")
def mgmod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_14117_amd import mg
    mg.lib()
    return mg


@pytest.fixture(scope="module")
def pools(mgmod):
    cls = env_classes(POOL, "bernoulli", 401)
    x0 = initial_state(POOL, D, 402)
    x0[19:, cls == 0] = 0
    mult = param_multipliers(POOL, 0.2, 403)
    act = actions(LMAX, NMAX, POOL, 404)
    return {"cls": cls, "x0": x0, "mult": mult, "act": act,
            "x0_d": dev(x0), "mult_d": dev(mult), "act_d": dev(act)}


def _req(pools, off, n, L):
    """Pointers into the pools: columns [off, off + n), row stride POOL."""
    return dict(n_envs=n, n_steps=L, x0_ptr=pools["x0_d"].data_ptr() + 4 * off,
                actions_ptr=pools["act_d"].data_ptr() + 4 * off, ld=POOL,
                env_class=pools["cls"][off:off + n], mult_ptr=pools["mult_d"].data_ptr() + 4 * off)


def _serve(srv, pools, reqs):
    outs, tickets = [], []
    for off, n, L in reqs:
        out = np.zeros((D, n), np.float32)
        st, t = srv.submit(out=out, **_req(pools, off, n, L))
        assert st == 0
        outs.append(out)
        tickets.append(t)
    lat = []
    for t in tickets:
        st, l = srv.wait(t, timeout_us=60_000_000)
        assert st == 0
        lat.append(l)
    return outs, lat


R = (1234, 1000, 20)     # the request that is checked alone and in the mix


def test_malformed_requests_refused_and_a_one_env_step_served(mgmod, pools):
    """Malformed requests (no envs, no steps, a row stride below the env count, a class
    the server does not have, no throttles and no seed) are refused with MG_ERR_INVALID
    before anything is queued (none counts as rejected for the cap); then the smallest
    request, one env for one control step, is served and equals mg_step bitwise."""
    from paper_2410_14117_amd.mg import MG_ERR_INVALID
    srv = mgmod.Server(CLASSES, DT, S)
    say("serve malformed requests")
    bad = [dict(_req(pools, 0, 5, 1), n_envs=0), dict(_req(pools, 0, 5, 1), n_steps=0),
           dict(_req(pools, 0, 5, 1), ld=4), dict(_req(pools, 0, 5, 1), actions_ptr=0),
           dict(_req(pools, 0, 5, 1), env_class=np.array([0, 1, 2, 0, 1]))]
    for kw in bad:
        n = kw["n_envs"]
        out = np.zeros((D, max(n, 1)), np.float32)
        if n == 0:
            kw = dict(kw, env_class=None)
            out = np.zeros((D, 0), np.float32)
        assert srv.submit(out=out, **kw)[0] == MG_ERR_INVALID, kw
    st = srv.stats()
    assert st["queued"] == 0 and st["completed"] == 0 and st["rejected"] == 0
    off = 777
    out = np.zeros((D, 1), np.float32)
    stt, t = srv.submit(out=out, **_req(pools, off, 1, 1))
    assert stt == 0 and srv.wait(t, 60_000_000)[0] == 0
    srv.close()
    sim = mgmod.Sim(CLASSES, 1, DT, S, env_class=pools["cls"][off:off + 1])
    sim.reset(state=dev(pools["x0"][:, off:off + 1]), param_mult=dev(pools["mult"][:, off:off + 1]))
    sim.step(dev(pools["act"][:1, :, off:off + 1]))
    np.testing.assert_array_equal(host(sim.get_state()), out)
    sim.close()


def test_alone_equals_mix_equals_step_and_oracle(mgmod, pools, oracle):
    say("serve alone")
    srv = mgmod.Server(CLASSES, DT, S)
    (alone,), _ = _serve(srv, pools, [R])
    say("serve mix")
    rng = np.random.default_rng(5)
    mix = []
    for k in range(30):
        n = int(np.exp(rng.uniform(np.log(16), np.log(20000))))
        off = int(rng.integers(0, POOL - n))
        mix.append((off, n, int(rng.integers(1, LMAX + 1))))
    mix.insert(12, R)
    outs, _ = _serve(srv, pools, mix)
    np.testing.assert_array_equal(outs[12], alone)
    st = srv.stats()
    assert st["completed"] == 32 and st["max_active_envs"] > R[1]
    srv.close()
    # the same request through mg_step (one fused launch of 20 control steps)
    off, n, L = R
    cls = pools["cls"][off:off + n]
    sim = mgmod.Sim(CLASSES, n, DT, S, env_class=cls)
    sim.reset(state=dev(pools["x0"][:, off:off + n]), param_mult=dev(pools["mult"][:, off:off + n]))
    sim.step(dev(pools["act"][:L, :, off:off + n]))
    np.testing.assert_array_equal(host(sim.get_state()), alone)
    sim.close()
    # and the FP64 oracle
    ref = oracle.rollout(CLASSES, pools["x0"][:, off:off + n], pools["act"][:L, :, off:off + n], S,
                         DT, env_class=cls, mult=pools["mult"][:, off:off + n])
    assert rel_err(alone, ref["x"]) <= TOL_TRAJ


def test_fifo_plain_baseline_same_results(mgmod, pools):
    """The baseline runs the plain per-sub-step kernel: equal to rounding (<= 1e-5)."""
    say("serve fifo")
    reqs = [R, (50, 300, 7), (9000, 4100, 3)]
    a = mgmod.Server(CLASSES, DT, S)
    outs_a, _ = _serve(a, pools, reqs)
    a.close()
    b = mgmod.Server(CLASSES, DT, S, fifo_plain=True)
    outs_b, _ = _serve(b, pools, reqs)
    b.close()
    for u, v in zip(outs_a, outs_b):
        assert rel_err(v, u) <= 1e-5


@pytest.mark.parametrize("K", [8, 64])
def test_steps_per_tick_same_results(mgmod, pools, K):
    """Pages advanced by up to K control steps per tick (as many as their request has left)
    end in the same states, bitwise, as with one step per tick: requests of 1 to 64 steps,
    most not a multiple of K, joining while others run; the same env-steps in fewer ticks."""
    say("serve steps per tick", K)
    reqs = [R, (50, 300, 7), (9000, 4100, 3), (20000, 700, 64), (15000, 2000, 1),
            (30000, 64, 9), (31000, 65, 17), (33000, 3000, 63)]
    a = mgmod.Server(CLASSES, DT, S)
    outs_a, _ = _serve(a, pools, reqs)
    st_a = a.stats()
    a.close()
    b = mgmod.Server(CLASSES, DT, S, steps_per_tick=K)
    outs_b, _ = _serve(b, pools, reqs)
    st_b = b.stats()
    b.close()
    for u, v in zip(outs_a, outs_b):
        np.testing.assert_array_equal(u, v)
    assert st_a["env_steps"] == st_b["env_steps"] == sum(n * L for _, n, L in reqs)
    assert st_b["ticks"] < st_a["ticks"]


def test_other_class_instantiations(mgmod, pools):
    """A server of three classes with 5 thrusters without lag, 7 with lag and 2 with lag
    (instantiations of the tick kernel the other tests leave out): each request's states
    equal those of mg_step, bitwise."""
    base = vehicle_variant(BLUEROV2_HEAVY, thr_map=1, thr_tau=0.05)
    classes = []
    for n_thr, tau in ((5, 0.0), (7, 0.05), (2, 0.05)):
        v = dict(base)
        v["thr_pos"] = v["thr_pos"][:n_thr]
        v["thr_dir"] = v["thr_dir"][:n_thr]
        v["thr_tau"] = tau
        classes.append(v)
    n = 3000
    cls = (np.arange(n) * 7 % 3).astype(np.int32)
    x0 = initial_state(n, 20, 411)
    x0[13:, cls == 0] = 0
    x0[15:, cls == 2] = 0
    act = actions(12, 7, n, 412)
    mult = param_multipliers(n, 0.2, 413)
    x0_d, act_d, mult_d = dev(x0), dev(act), dev(mult)
    say("serve three classes")
    srv = mgmod.Server(classes, DT, S, steps_per_tick=4)
    outs = []
    for L, lo, hi in ((12, 0, 1000), (5, 1000, 3000)):
        out = np.zeros((20, hi - lo), np.float32)
        st, t = srv.submit(hi - lo, L, x0_d.data_ptr() + 4 * lo, act_d.data_ptr() + 4 * lo, n, out,
                           env_class=cls[lo:hi], mult_ptr=mult_d.data_ptr() + 4 * lo)
        assert st == 0
        outs.append((t, out, L, lo, hi))
    for t, out, L, lo, hi in outs:
        assert srv.wait(t, 60_000_000)[0] == 0
        sim = mgmod.Sim(classes, hi - lo, DT, S, env_class=cls[lo:hi])
        sim.reset(state=dev(x0[:, lo:hi]), param_mult=dev(mult[:, lo:hi]))
        sim.step(dev(act[:L, :, lo:hi]))
        np.testing.assert_array_equal(host(sim.get_state()), out)
        sim.close()
    srv.close()


def test_memory_cap_admission(mgmod, pools):
    """A 20-page cap: requests wait for pages instead of failing; a request larger than the
    whole cap is rejected at submit; no more pages than the cap are ever created."""
    say("serve cap")
    pb = mgmod.page_bytes(D)
    srv = mgmod.Server(CLASSES, DT, S, mem_cap_bytes=20 * pb)
    big = np.zeros((D, 3000), np.float32)
    st, _ = srv.submit(out=big, **_req(pools, 0, 3000, 2))     # >= 47 pages
    assert st == 1
    reqs = [(k * 500, 400, 6) for k in range(8)]                # ~8 pages each
    outs, _ = _serve(srv, pools, reqs)
    s = srv.stats()
    assert s["completed"] == 8 and s["rejected"] == 1
    assert s["created_pages"] <= 20 and s["cap_pages"] == 20
    srv.close()
    ref = mgmod.Server(CLASSES, DT, S)
    outs_ref, _ = _serve(ref, pools, reqs)
    ref.close()
    for u, v in zip(outs, outs_ref):
        np.testing.assert_array_equal(u, v)


def test_reserved_pages_are_created_up_front(mgmod, pools):
    """reserve_bytes creates page memory at start (capped at the cap); admissions within it
    create no pages; results equal those of an on-demand server bitwise."""
    say("serve reserve")
    pb = mgmod.page_bytes(D)
    srv = mgmod.Server(CLASSES, DT, S, mem_cap_bytes=3000 * pb, reserve_bytes=2100 * pb)
    s0 = srv.stats()
    assert s0["created_pages"] >= 2100 and s0["created_pages"] <= 3000
    reqs = [(k * 4000, 3000, 5) for k in range(6)]          # ~50 pages each
    outs, _ = _serve(srv, pools, reqs)
    s1 = srv.stats()
    assert s1["created_pages"] == s0["created_pages"] and s1["completed"] == 6
    srv.close()
    capped = mgmod.Server(CLASSES, DT, S, mem_cap_bytes=40 * pb, reserve_bytes=10 ** 9)
    assert capped.stats()["created_pages"] == 40
    capped.close()
    with pytest.raises(mgmod.MgError):
        mgmod.Server(CLASSES, DT, S, reserve_bytes=-1)
    ref = mgmod.Server(CLASSES, DT, S)
    outs_ref, _ = _serve(ref, pools, reqs)
    ref.close()
    for u, v in zip(outs, outs_ref):
        np.testing.assert_array_equal(u, v)


def test_request_joins_mid_flight(mgmod, pools):
    """A short request submitted while a long one runs finishes first (continuous batching)."""
    say("serve join")
    srv = mgmod.Server(CLASSES, DT, S)
    long_out = np.zeros((D, 30000), np.float32)
    st, t_long = srv.submit(out=long_out, **_req(pools, 0, 30000, 64))
    assert st == 0
    t0 = time.time()
    while srv.stats()["active_envs"] == 0 and time.time() - t0 < 30:
        pass
    short_out = np.zeros((D, 100), np.float32)
    st, t_short = srv.submit(out=short_out, **_req(pools, 35000, 100, 1))
    assert st == 0
    assert srv.wait(t_short, 60_000_000)[0] == 0
    still_running = srv.wait(t_long, 0)[0] == 5          # MG_ERR_BUSY
    assert srv.wait(t_long, 60_000_000)[0] == 0
    assert still_running
    srv.close()


def test_poisson_clients_all_complete(mgmod, pools):
    """8 client threads, Poisson arrivals (aggregate 400 req/s for 0.5 s), log-uniform env
    counts in [16, 4096], rollout lengths uniform in [1, 64]."""
    say("serve poisson")
    srv = mgmod.Server(CLASSES, DT, S)
    rng = np.random.default_rng(9)
    results = []
    lock = threading.Lock()
    t_start = mgmod.Server.clock_ns() + 20_000_000

    def client(seed):
        r = np.random.default_rng(seed)
        t = t_start
        while True:
            t += int(r.exponential(1.0 / 50.0) * 1e9)
            if t > t_start + 500_000_000:
                break
            n = int(np.exp(r.uniform(np.log(16), np.log(4096))))
            L = int(r.integers(1, 65))
            off = int(r.integers(0, POOL - n))
            while mgmod.Server.clock_ns() < t:
                time.sleep(0.0002)
            out = np.zeros((D, n), np.float32)
            st, tk = srv.submit(out=out, arrival_ns=t, **_req(pools, off, n, L))
            with lock:
                results.append((st, tk, out))

    ths = [threading.Thread(target=client, args=(100 + i,)) for i in range(8)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    lats = []
    for st, tk, out in results:
        assert st == 0
        st2, lat = srv.wait(tk, 60_000_000)
        assert st2 == 0
        lats.append(lat)
        assert np.isfinite(out).all()
    assert len(lats) > 100
    assert srv.stats()["completed"] == len(lats)
    srv.close()
    assert 0 < np.percentile(lats, 50) <= np.percentile(lats, 99) < 30
    assert rng is not None


@pytest.mark.slow
def test_c5_trace_in_the_benchmark_configuration(mgmod):
    """The benchmark's serving configuration (8 control steps per tick, 2 GiB reserved, 32
    Poisson clients at 2000 req/s for 0.3 s, env counts log-uniform in [16, 65536], half step
    requests and half rollouts of 1..64 steps, mixed classes): every request completes with
    finite states, and 12 of them (the largest, the longest and 10 at random) equal mg_step's
    result bitwise."""
    P = 1 << 17
    cls = env_classes(P, "bernoulli", 421)
    x0 = initial_state(P, D, 422)
    x0[19:, cls == 0] = 0
    mult = param_multipliers(P, 0.2, 423)
    act = actions(LMAX, NMAX, P, 424)
    x0_d, mult_d, act_d = dev(x0), dev(mult), dev(act)
    rng = np.random.default_rng(425)
    trace = []
    for k in range(32):
        t = 0.0
        while True:
            t += rng.exponential(32 / 2000.0)
            if t > 0.3:
                break
            n = int(round(np.exp(rng.uniform(np.log(16), np.log(65536)))))
            L = 1 if rng.random() < 0.5 else int(rng.integers(1, LMAX + 1))
            trace.append((t, n, L, int(rng.integers(0, P - n + 1))))
    trace.sort()
    say(f"serve c5 configuration, {len(trace)} requests")
    srv = mgmod.Server(CLASSES, DT, S, steps_per_tick=8, reserve_bytes=2 << 30)
    t0 = mgmod.Server.clock_ns() + 20_000_000
    subs = []
    for t, n, L, off in trace:
        at = t0 + int(t * 1e9)
        while mgmod.Server.clock_ns() < at:
            time.sleep(0.0002)
        out = np.zeros((D, n), np.float32)
        st, tk = srv.submit(n, L, x0_d.data_ptr() + 4 * off, act_d.data_ptr() + 4 * off, P, out,
                            env_class=cls[off:off + n], mult_ptr=mult_d.data_ptr() + 4 * off,
                            arrival_ns=at)
        assert st == 0
        subs.append((tk, out, n, L, off))
    for tk, out, n, L, off in subs:
        assert srv.wait(tk, 60_000_000)[0] == 0
        assert np.isfinite(out).all()
    srv.close()
    pick = {int(np.argmax([s[2] for s in subs])), int(np.argmax([s[3] for s in subs]))}
    pick |= set(int(i) for i in rng.choice(len(subs), 10, replace=False))
    for i in sorted(pick):
        _, out, n, L, off = subs[i]
        c = cls[off:off + n]
        sim = mgmod.Sim(CLASSES, n, DT, S, env_class=c)
        sim.reset(state=dev(x0[:, off:off + n]), param_mult=dev(mult[:, off:off + n]))
        sim.step(dev(act[:L, :, off:off + n]))
        np.testing.assert_array_equal(host(sim.get_state()), out)
        sim.close()


def test_seed_mode_equals_pointer_mode(mgmod, pools):
    """Requests whose throttles the tick kernel generates from a seed (SplitMix64) give,
    bitwise, the final states of the same requests with those throttles generated on the
    host and passed by pointer; 12 requests of both classes, 1 to 64 control steps, served
    together in each mode at 8 control steps per tick."""
    rng = np.random.default_rng(431)
    reqs = []
    for k in range(12):
        n = int(np.exp(rng.uniform(np.log(16), np.log(6000))))
        reqs.append((int(rng.integers(0, POOL - n)), n, int(rng.integers(1, LMAX + 1)),
                     int(rng.integers(0, 2 ** 63)) * 2 + 1))
    srv = mgmod.Server(CLASSES, DT, S, steps_per_tick=8)
    say("serve seed mode: 12 requests, throttles generated on the device")
    seeded, tickets = [], []
    for off, n, L, seed in reqs:
        out = np.zeros((D, n), np.float32)
        r = _req(pools, off, n, L)
        r["actions_ptr"] = 0
        st, t = srv.submit(out=out, action_seed=seed, **r)
        assert st == 0
        seeded.append(out)
        tickets.append(t)
    for t in tickets:
        assert srv.wait(t, 60_000_000)[0] == 0
    say("serve pointer mode: the same throttles generated on the host")
    keep, tickets, ptr = [], [], []
    for off, n, L, seed in reqs:
        a = dev(splitmix64_throttles(seed, L, NMAX, n))
        keep.append(a)
        out = np.zeros((D, n), np.float32)
        # the host throttles have column stride n, so x0 and the multipliers are passed
        # as copies of the request's columns with that stride too
        x0c = dev(pools["x0"][:, off:off + n])
        mc = dev(pools["mult"][:, off:off + n])
        keep += [x0c, mc]
        st, t = srv.submit(n, L, x0c.data_ptr(), a.data_ptr(), n, out,
                           env_class=pools["cls"][off:off + n], mult_ptr=mc.data_ptr())
        assert st == 0
        ptr.append(out)
        tickets.append(t)
    for t in tickets:
        assert srv.wait(t, 60_000_000)[0] == 0
    srv.close()
    for a, b in zip(seeded, ptr):
        assert np.isfinite(a).all()
        np.testing.assert_array_equal(a, b)


def test_two_waiters_on_one_ticket(mgmod, pools):
    """Two threads wait on one ticket: exactly one receives the result (MG_OK), the other
    MG_ERR_INVALID (the ticket was consumed), neither blocks for ever."""
    srv = mgmod.Server(CLASSES, DT, S)
    out = np.zeros((D, 3000), np.float32)
    say("serve two waiters on one ticket")
    st, tk = srv.submit(out=out, **_req(pools, 100, 3000, 64))
    assert st == 0
    got = []
    lock = threading.Lock()

    def waiter():
        r = srv.wait(tk, 60_000_000)[0]
        with lock:
            got.append(r)

    ths = [threading.Thread(target=waiter) for _ in range(2)]
    for th in ths:
        th.start()
    for th in ths:
        th.join(90)
    assert sorted(got) == [0, 1]
    srv.close()


def test_injected_tick_failure_fails_every_request_in_flight(mgmod, pools, monkeypatch):
    """With MG_SERVER_FAIL_TICK=3 the scheduler treats its third tick's completion as a
    device error (set on the host; nothing faults on the GPU): every request not yet
    delivered completes with MG_ERR_DEVICE, none hangs, later submits are refused with
    MG_ERR_DEVICE, and the server still shuts down cleanly."""
    monkeypatch.setenv("MG_SERVER_FAIL_TICK", "3")
    srv = mgmod.Server(CLASSES, DT, S)
    monkeypatch.delenv("MG_SERVER_FAIL_TICK")
    say("serve injected failure at tick 3: 10 rollouts of 64 steps")
    subs = []
    for k in range(10):
        out = np.zeros((D, 500), np.float32)
        st, tk = srv.submit(out=out, **_req(pools, 600 * k, 500, 64))
        assert st == 0
        subs.append(tk)
    res = [srv.wait(tk, 60_000_000)[0] for tk in subs]
    assert set(res) == {3}                       # MG_ERR_DEVICE, all of them (64 > 3 ticks)
    out = np.zeros((D, 16), np.float32)
    assert srv.submit(out=out, **_req(pools, 0, 16, 1))[0] == 3
    assert "injected" in srv.last_error()
    srv.close()


def test_native_clients_replay(mgmod, pools):
    """32 native client threads (libmg_clients.so) replay a 0.4 s Poisson trace at 2000
    req/s with seed-generated throttles, submitting concurrently: every request completes
    with finite states, latencies are positive, and two of the requests equal, bitwise, the
    same requests served alone afterwards."""
    rng = np.random.default_rng(441)
    reqs = []
    for k in range(32):
        t = 0.0
        while True:
            t += rng.exponential(32 / 2000.0)
            if t > 0.4:
                break
            n = int(round(np.exp(rng.uniform(np.log(16), np.log(8192)))))
            L = 1 if rng.random() < 0.5 else int(rng.integers(1, LMAX + 1))
            off = int(rng.integers(0, POOL - n + 1))
            reqs.append({"client": k, "at_ns": int(t * 1e9), "n_envs": n, "n_steps": L,
                         "x0_ptr": pools["x0_d"].data_ptr() + 4 * off, "ld": POOL,
                         "out": np.zeros((D, n), np.float32),
                         "env_class": pools["cls"][off:off + n],
                         "mult_ptr": pools["mult_d"].data_ptr() + 4 * off,
                         "action_seed": int(rng.integers(0, 2 ** 63)), "off": off})
    srv = mgmod.Server(CLASSES, DT, S, steps_per_tick=8)
    say(f"serve native replay: {len(reqs)} requests from 32 client threads")
    status, lat, lag, _ = srv.replay(reqs, 32)
    assert (status == 0).all() and (lat > 0).all()
    for q in reqs:
        assert np.isfinite(q["out"]).all()
    for q in (reqs[0], reqs[len(reqs) // 2]):
        out = np.zeros_like(q["out"])
        st, tk = srv.submit(q["n_envs"], q["n_steps"], q["x0_ptr"], 0, POOL, out,
                            env_class=q["env_class"], mult_ptr=q["mult_ptr"],
                            action_seed=q["action_seed"])
        assert st == 0 and srv.wait(tk, 60_000_000)[0] == 0
        np.testing.assert_array_equal(out, q["out"])
    assert srv.stats()["completed"] == len(reqs) + 2
    srv.close()


def test_reserved_staging_defers_instead_of_growing(mgmod):
    """A server reserved with 4096 pages (4096 pages of join and leave staging per tick,
    result buffers of 2^22 floats, 32 sub-steps per control step, 64 control steps per
    tick).  A blocker of 190 000 envs x 64 control steps (about 3000 pages, 4.0e6 result
    floats: within the staging) keeps the GPU busy for a few milliseconds while six
    requests of 50 000 envs x 1 step queue up: five join together (about 3910 pages), the
    sixth waits for the next tick (join staging full), and of the five, which all finish in
    that tick, three retire at once and the others a tick later (results beyond 2^22
    floats).  No staging grows, and every result equals, bitwise, the same request served
    alone on an unreserved server."""
    P, n, S32 = 1 << 18, 50000, 32
    cls = env_classes(P, "bernoulli", 451)
    x0 = initial_state(P, D, 452)
    x0[19:, cls == 0] = 0
    x0_d, mult_d = dev(x0), dev(param_multipliers(P, 0.2, 453))
    offs = [7919 * k for k in range(6)]

    def submit(srv, off, m, L, seed):
        out = np.zeros((D, m), np.float32)
        st, tk = srv.submit(m, L, x0_d.data_ptr() + 4 * off, 0, P, out,
                            env_class=cls[off:off + m], mult_ptr=mult_d.data_ptr() + 4 * off,
                            action_seed=seed)
        assert st == 0
        return tk, out

    srv = mgmod.Server(CLASSES, DT / 8, S32, steps_per_tick=64,
                       reserve_bytes=4096 * mgmod.page_bytes(D))
    s0 = srv.stats()
    say("serve reserved staging: blocker of 190000 envs, then 6 x 50000 envs")
    tb, _ = submit(srv, 0, 190000, 64, 1)
    while srv.stats()["ticks"] == s0["ticks"]:
        pass
    subs = [submit(srv, off, n, 1, 100 + k) for k, off in enumerate(offs)]
    assert srv.wait(tb, 60_000_000)[0] == 0
    for tk, _ in subs:
        assert srv.wait(tk, 60_000_000)[0] == 0
    s1 = srv.stats()
    srv.close()
    assert s1["grow_events"] == s0["grow_events"]
    assert s1["held_joins"] > s0["held_joins"]
    assert s1["deferred_retires"] > s0["deferred_retires"]
    ref = mgmod.Server(CLASSES, DT / 8, S32, steps_per_tick=64)
    for k, off in enumerate(offs):
        tk, out = submit(ref, off, n, 1, 100 + k)
        assert ref.wait(tk, 60_000_000)[0] == 0
        np.testing.assert_array_equal(out, subs[k][1])
    ref.close()


def test_cancel_queued_and_admitted_requests(mgmod, pools):
    """A server capped at A's pages plus 10 (256 sub-steps per control step, one control
    step per tick): A (40 000 envs x 64 steps) is admitted, B (2000 envs) waits for pages
    and C (300 envs) waits behind B (FIFO admission).  Cancelling C takes it out of the
    queue at once; cancelling A retires it at the next tick without delivery (its output
    stays as the client left it); both complete with MG_ERR_CANCELLED.  B then runs on the
    freed pages and its result equals, bitwise, B served alone.  A completed ticket cannot
    be cancelled."""
    from paper_2410_14117_amd.mg import MG_ERR_CANCELLED, MG_ERR_INVALID
    page = mgmod.page_bytes(D)
    c = pools["cls"][:40000]
    pages_a = -(-int((c == 0).sum()) // 64) - (-int((c == 1).sum()) // 64)
    S256, dt = 256, DT / 64
    srv = mgmod.Server(CLASSES, dt, S256, mem_cap_bytes=(pages_a + 10) * page)
    outs = {k: np.full((D, n), -7.0, np.float32) for k, n in (("A", 40000), ("B", 2000),
                                                               ("C", 300))}
    say("serve cancel: A admitted, B and C queued")
    st, ta = srv.submit(out=outs["A"], **_req(pools, 0, 40000, 64))
    assert st == 0
    t0 = time.time()
    while srv.stats()["active_envs"] == 0 and time.time() - t0 < 30:
        pass
    st, tb = srv.submit(out=outs["B"], **_req(pools, 100, 2000, 5))
    assert st == 0
    st, tc = srv.submit(out=outs["C"], **_req(pools, 5000, 300, 5))
    assert st == 0
    assert srv.stats()["queued"] == 2
    assert srv.cancel(tc) == 0
    assert srv.cancel(ta) == 0
    assert srv.wait(tc, 60_000_000)[0] == MG_ERR_CANCELLED
    assert srv.wait(ta, 60_000_000)[0] == MG_ERR_CANCELLED
    assert srv.wait(tb, 60_000_000)[0] == 0
    assert (outs["A"] == -7.0).all() and (outs["C"] == -7.0).all()
    assert srv.cancel(tb) == MG_ERR_INVALID and srv.cancel(12345678) == MG_ERR_INVALID
    st = srv.stats()
    assert st["queued"] == 0 and st["completed"] == 1
    srv.close()
    ref = mgmod.Server(CLASSES, dt, S256)
    alone = np.zeros((D, 2000), np.float32)
    st, t = ref.submit(out=alone, **_req(pools, 100, 2000, 5))
    assert st == 0 and ref.wait(t, 60_000_000)[0] == 0
    ref.close()
    np.testing.assert_array_equal(outs["B"], alone)
