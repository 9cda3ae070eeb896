"""GPU: snapshots at output times and the maximum-depth map (Section 3, the
run writes the state at chosen output times), against the FP64 checker and
bitwise against plain reads of the same run."""
import sys

import numpy as np
import pytest

import oracle
from parity import TOL_SHOCK, assert_front_parity, rel_l2
from paper_2301_12010_amd import inputs, swe

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def step_times(sc, n):
    o = oracle.Oracle.from_scenario(sc)
    t = []
    for _ in range(n):
        assert o.step(1) == 0
        t.append(o.scalars()["t"])
    return t


def test_outputs_and_max_depth_against_checker():
    sc = inputs.nwave_beach(nx=512, ny=64, dx=8.0)
    n = 60
    t = step_times(sc, n)
    # between the ends of steps 10|11, 25|26 (twice: one step serves both),
    # 59|60, and one time the run never reaches
    times = [0.5 * (t[9] + t[10]), 0.5 * (t[24] + t[25]), 0.4 * t[24] + 0.6 * t[25],
             0.5 * (t[58] + t[59]), 10.0 * t[-1]]
    o = oracle.Oracle.from_scenario(sc)
    ref, ref_hmax = o.run_with_outputs(n, times, max_depth=True)

    s = swe.Solver.from_scenario(sc)
    s.set_option(swe.OPT_GRAPH_STEPS, 16)
    s.set_outputs(times)
    s.track_max_depth(True)
    got = [None] * len(times)
    for chunk in range(3):
        s.step(20)
        for k in range(len(times)):  # non-blocking polls while steps run
            if got[k] is None:
                got[k] = s.output(k, wait=False)
    for k in range(len(times)):
        if got[k] is None:
            got[k] = s.output(k, wait=True)
    hmax = s.max_depth()
    st = s.read()[3]
    s.close()
    assert st["step"] == n
    assert got[4] is None and ref[4] is None
    for k in range(4):
        g, r = got[k], ref[k]
        assert g[4] == r[4], (k, g[4], r[4])
        assert abs(g[3] - r[3]) <= 1e-6 * r[3]
        assert_front_parity(g, r, TOL_SHOCK, f"output {k} step {g[4]}")
    assert all(np.array_equal(a, b) for a, b in zip(got[1][:3], got[2][:3]))
    e = rel_l2(hmax, ref_hmax)
    say("max depth", e, float(np.abs(hmax - ref_hmax).max()))
    assert e <= TOL_SHOCK
    assert np.all(hmax >= sc.h)


def test_outputs_and_max_depth_bitwise_against_plain_reads():
    sc = inputs.random_wet(150, 70, seed=7, dry_fraction=0.05)
    n = 24
    t = step_times(sc, n)
    times = [0.5 * (t[2] + t[3]), 0.5 * (t[12] + t[13]), 0.5 * (t[22] + t[23])]
    s = swe.Solver.from_scenario(sc)
    s.set_option(swe.OPT_GRAPH_STEPS, 5)
    s.set_outputs(times)
    s.track_max_depth(True)
    s.step(n)
    snaps = [s.output(k, wait=True) for k in range(len(times))]
    hmax = s.max_depth()
    s.close()

    plain = swe.Solver.from_scenario(sc)
    run_max = sc.h.astype(np.float32).copy()
    by_step = {}
    for k in range(1, n + 1):
        plain.step(1)
        h, hu, hv, st = plain.read()
        np.maximum(run_max, h, out=run_max)
        by_step[k] = (h, hu, hv, st["t"])
    plain.close()
    for snap in snaps:
        assert snap is not None
        h, hu, hv, tk, step = snap
        rh, rhu, rhv, rt = by_step[step]
        assert tk == rt
        assert np.array_equal(h, rh) and np.array_equal(hu, rhu) and np.array_equal(hv, rhv)
    # t[i] ends step i + 1: the midpoints are first reached by steps 4, 14, 24
    assert [sn[4] for sn in snaps] == [4, 14, 24]
    assert np.array_equal(hmax, run_max)


def test_output_requests_validated_and_replaced():
    sc = inputs.random_wet(40, 30, seed=8)
    s = swe.Solver.from_scenario(sc)
    for bad in ([1.0, 0.5], [float("nan")], [float("inf")]):
        with pytest.raises(swe.SweError) as ei:
            s.set_outputs(bad)
        assert ei.value.code == swe.EINVAL
    with pytest.raises(swe.SweError):
        s.max_depth()  # not tracking
    s.set_outputs([0.0])      # reached by the first step
    s.set_outputs([1e-9, 1e9])  # replaces the request
    s.step(3)
    first = s.output(0, wait=True)
    assert first is not None and first[4] == 1
    assert s.output(1, wait=True) is None
    with pytest.raises(swe.SweError):
        s.output(2)
    s.set_outputs([])  # cleared: no output index is valid
    with pytest.raises(swe.SweError):
        s.output(0)
    s.track_max_depth(True)
    s.track_max_depth(False)
    with pytest.raises(swe.SweError):
        s.max_depth()
    s.step(2)
    assert s.read()[3]["step"] == 5
    s.close()


@pytest.mark.parametrize("mode", [swe.BATCH_ROUNDS, swe.BATCH_PERSISTENT])
def test_batch_max_depth_equals_alone(mode):
    # maximum-depth maps of ensemble members kept inside the batch's launches
    mix = [(inputs.random_wet(130, 70, seed=11, dry_fraction=0.05), 9),
           (inputs.nwave_beach(nx=256, ny=32, dx=8.0), 12),
           (inputs.random_wet(40, 24, seed=12), 0)]
    bt = swe.Batch()
    bt.set_mode(mode, True)
    for i, (sc, n) in enumerate(mix):
        bt.add_scenario(sc, n)
        if i != 1:
            bt.track_max_depth(i)
    bt.track_max_depth(1)   # also on the last one, then restarted below
    bt.track_max_depth(1, False)
    bt.track_max_depth(1, True)
    bt.run(4)
    bt.run()
    for i, (sc, n) in enumerate(mix):
        s = swe.Solver.from_scenario(sc)
        s.track_max_depth(True)
        s.step(n)
        ref = s.max_depth()
        s.close()
        got = bt.max_depth(i)
        assert np.array_equal(got, ref), i
    assert np.array_equal(bt.max_depth(2), mix[2][0].h)  # no steps: the start
    bt.track_max_depth(0, False)
    with pytest.raises(swe.SweError):
        bt.max_depth(0)
    bt.close()


def test_outputs_reach_the_host_by_non_blocking_polls_alone():
    # many back-to-back swe_step calls keep both metadata copies in flight;
    # the copies they owe are made by later polls, so polling without waiting
    # delivers a snapshot taken in the last steps
    import time
    sc = inputs.random_wet(64, 48, seed=13)
    t = step_times(sc, 30)
    s = swe.Solver.from_scenario(sc)
    s.set_outputs([0.5 * (t[27] + t[28])])
    for _ in range(30):
        s.step(1)
    got, deadline = None, time.time() + 30.0
    while got is None and time.time() < deadline:
        got = s.output(0, wait=False)
        time.sleep(0.001)
    assert got is not None and got[4] == 29
    h, hu, hv, st = s.read()
    s.close()
    ref = swe.Solver.from_scenario(sc)
    ref.step(29)
    rh = ref.read()
    ref.close()
    assert all(np.array_equal(a, b) for a, b in zip(got[:3], rh[:3]))


def test_timed_steps_take_outputs_like_plain_steps():
    # the measurement call advances the state like swe_step: the snapshot and
    # the maximum-depth map equal those of the same steps taken plainly
    sc = inputs.random_wet(64, 48, seed=14)
    t = step_times(sc, 10)
    times = [0.5 * (t[4] + t[5])]
    runs = []
    for timed in (True, False):
        s = swe.Solver.from_scenario(sc)
        s.set_outputs(times)
        s.track_max_depth(True)
        if timed:
            s.time_stages(10)
        else:
            s.step(10)
        runs.append((s.output(0, wait=True), s.max_depth(), s.read()))
        s.close()
    (snap_a, hmax_a, st_a), (snap_b, hmax_b, st_b) = runs
    assert snap_a is not None and snap_a[4] == snap_b[4] == 6
    assert all(np.array_equal(a, b) for a, b in zip(snap_a[:3], snap_b[:3]))
    assert np.array_equal(hmax_a, hmax_b)
    assert all(np.array_equal(a, b) for a, b in zip(st_a[:3], st_b[:3]))
    assert st_a[3]["step"] == 10
