"""GPU: the continuous-batching server.  Results equal the same scenarios run
alone, admission respects the memory budget, failures stay isolated, and
cancellation works."""
import sys
import time

import numpy as np
import pytest

from paper_2301_12010_amd import inputs, swe

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def alone(sc, n):
    s = swe.Solver.from_scenario(sc)
    s.set_option(swe.OPT_TILE, 1)
    s.step(n)
    out = s.read()
    s.close()
    return out


def wait_all(sv, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t in out:
                continue
            r, st = sv.poll(t)
            if r["status"] != swe.PENDING:
                out[t] = (r, st)
        assert time.time() - t0 < timeout, "server did not finish in time"
        time.sleep(0.002)
    return out


def test_results_equal_alone_with_staggered_arrivals():
    mix = [(inputs.random_wet(64, 48, seed=11), 23), (inputs.random_wet(130, 70, seed=12), 17),
           (inputs.dam_break(nx=128, ny=64), 40), (inputs.random_wet(33, 17, seed=13), 9),
           (inputs.parabolic_bowl(nx=150, ny=9, dx=4.0), 31)]
    sv = swe.Server(mem_budget=256 << 20, max_slots=8, segment_steps=5)
    tickets = []
    for sc, n in mix:
        tickets.append(sv.submit_scenario(sc, n))
        time.sleep(0.01)  # later requests arrive while earlier ones run
    res = wait_all(sv, tickets)
    st = sv.stats()
    say("server stats", st)
    for t, (sc, n) in zip(tickets, mix):
        r, state = res[t]
        assert r["status"] == swe.DONE and r["steps"] == n
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        ref = alone(sc, n)
        for a, b in zip(state, ref[:3]):
            assert np.array_equal(a, b), sc.name
        assert r["t"] == ref[3]["t"]
    assert st["completed"] == len(mix) and st["segments"] >= 2
    sv.close()


def test_admission_by_memory_footprint():
    scen = [inputs.random_wet(256, 256, seed=20 + k) for k in range(6)]
    fp = swe.footprint(256, 256)
    budget = 2 * fp + fp // 2  # two resident scenarios at most
    sv = swe.Server(mem_budget=budget, max_slots=16, segment_steps=4)
    tickets = [sv.submit_scenario(sc, 12) for sc in scen]
    res = wait_all(sv, tickets)
    st = sv.stats()
    say("admission stats", st, "footprint", fp)
    assert st["mem_high_water"] <= budget
    assert st["mem_high_water"] <= 2 * ((fp + 255) // 256 * 256)
    admits = sorted(res[t][0]["t_admit"] for t in tickets)
    dones = sorted(res[t][0]["t_done"] for t in tickets)
    assert admits[2] >= dones[0]  # the third request had to wait for memory
    for t, sc in zip(tickets, scen):
        ref = alone(sc, 12)
        for a, b in zip(res[t][1], ref[:3]):
            assert np.array_equal(a, b)
    big = inputs.random_wet(1024, 1024, seed=3)
    with pytest.raises(swe.SweError) as ei:
        sv.submit_scenario(big, 1)
    assert ei.value.code == swe.ENOMEM
    sv.close()


def test_failures_are_isolated_and_cancel_works():
    from dataclasses import replace
    good = inputs.random_wet(64, 64, seed=31)
    bad = inputs.random_wet(64, 64, seed=32)
    bad = replace(bad, params=replace(bad.params, cfl=0.0, dt_fixed=50.0))
    sv = swe.Server(mem_budget=64 << 20, max_slots=8, segment_steps=3)
    nan_h = good.h.copy()
    nan_h[5, 5] = np.nan
    with pytest.raises(swe.SweError) as ei:
        sv.submit(good.params, good.b, good.n, nan_h, good.hu, good.hv, 5)
    assert ei.value.code == swe.EINVAL
    t_good = sv.submit_scenario(good, 30)
    t_bad = sv.submit_scenario(bad, 60)
    t_long = sv.submit_scenario(inputs.random_wet(64, 64, seed=33), 100000)
    time.sleep(0.05)
    sv.cancel(t_long)
    res = wait_all(sv, [t_good, t_bad, t_long])
    assert res[t_bad][0]["status"] == swe.FAILED and res[t_bad][0]["error"] == swe.ENONFINITE
    assert res[t_long][0]["status"] == swe.CANCELLED
    assert res[t_good][0]["status"] == swe.DONE
    ref = alone(good, 30)
    for a, b in zip(res[t_good][1], ref[:3]):
        assert np.array_equal(a, b)
    with pytest.raises(swe.SweError) as ei:
        sv.poll(t_good)  # released after its final status was reported
    assert ei.value.code == swe.ENOTFOUND
    sv.close()


@pytest.mark.parametrize("mode", [swe.BATCH_ROUNDS, swe.BATCH_PERSISTENT])
def test_served_maximum_depth_maps_equal_alone(mode):
    # requests that keep their inundation map next to ones that do not; each
    # map equals the single-scenario map of the same run, bitwise
    mix = [(inputs.nwave_beach(nx=256, ny=32, dx=8.0), 37, True),
           (inputs.random_wet(64, 48, seed=31, dry_fraction=0.05), 23, False),
           (inputs.random_wet(130, 70, seed=32, dry_fraction=0.05), 29, True),
           (inputs.random_wet(40, 24, seed=33), 0, True)]
    sv = swe.Server(mem_budget=256 << 20, max_slots=8, segment_steps=7)
    sv.set_mode(mode)
    tickets = []
    for sc, n, keep in mix:
        tickets.append(sv.submit_scenario(sc, n, max_depth=keep))
        time.sleep(0.005)
    # a map asked of a request that keeps none is refused without releasing it
    with pytest.raises(swe.SweError) as ei:
        sv.poll(tickets[1], want_max_depth=True)
    assert ei.value.code == swe.EINVAL
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t, (sc, n, keep) in zip(tickets, mix):
            if t in out:
                continue
            r, st = sv.poll(t, want_max_depth=keep)
            if r["status"] != swe.PENDING:
                out[t] = (r, st)
        assert time.time() - t0 < 60.0, "server did not finish in time"
        time.sleep(0.002)
    for t, (sc, n, keep) in zip(tickets, mix):
        r, state = out[t]
        assert r["status"] == swe.DONE and r["steps"] == n
        s = swe.Solver.from_scenario(sc)
        s.track_max_depth(True)
        s.step(n)
        ref = s.read()
        ref_max = s.max_depth()
        s.close()
        assert all(np.array_equal(a, b) for a, b in zip(state[:3], ref[:3])), sc.name
        if keep:
            assert len(state) == 4 and np.array_equal(state[3], ref_max), sc.name
        else:
            assert len(state) == 3
    # the map's plane is part of the footprint: nothing stays allocated
    assert sv.stats()["mem_in_use"] == 0
    sv.close()


def test_compensated_requests_equal_compensated_contexts():
    # SWE_OPT_COMPENSATED on a server (before the first submit): every
    # request's footprint carries its residual planes and the result equals a
    # context with the option, bitwise; after a submit the option is fixed
    mix = [(inputs.random_wet(64, 48, seed=21, dry_fraction=0.05), 13), (inputs.dam_break(nx=128, ny=64), 20)]
    sv = swe.Server(mem_budget=256 << 20, max_slots=8, segment_steps=5)
    sv.set_option(swe.OPT_COMPENSATED, 1)
    tickets = [sv.submit_scenario(sc, n) for sc, n in mix]
    with pytest.raises(swe.SweError) as ei:
        sv.set_option(swe.OPT_COMPENSATED, 0)
    assert ei.value.code == swe.EBUSY
    res = wait_all(sv, tickets)
    for t, (sc, n) in zip(tickets, mix):
        r, state = res[t]
        assert r["status"] == swe.DONE
        s = swe.Solver.from_scenario(sc)
        s.set_option(swe.OPT_TILE, 1)
        s.set_option(swe.OPT_COMPENSATED, 1)
        s.step(n)
        ref = s.read()
        s.close()
        for a, b in zip(state, ref[:3]):
            assert np.array_equal(a, b), sc.name
    sv.close()
