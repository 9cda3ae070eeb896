"""GPU: batched scenarios (one persistent launch, or one launch per round)
give each scenario exactly the state it reaches alone, and match the FP64
checker."""
import sys

import numpy as np
import pytest

import oracle
from parity import TOL_SHOCK, TOL_SMOOTH, assert_epilogue_parity, assert_front_parity, field_errors
from paper_2301_12010_amd import inputs, swe

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def alone(sc, nsteps, tile):
    s = swe.Solver.from_scenario(sc)
    s.set_option(swe.OPT_TILE, tile)
    s.step(nsteps)
    out = s.read()
    s.close()
    return out


def small_mix():
    return [
        (inputs.random_wet(64, 48, seed=1), 5),
        (inputs.random_wet(130, 70, seed=2, dry_fraction=0.05), 9),
        (inputs.random_wet(33, 17, seed=3), 3),
        (inputs.dam_break(nx=200, ny=100), 7),
        (inputs.random_wet(20, 20, seed=4), 0),
        (inputs.parabolic_bowl(nx=150, ny=9, dx=4.0), 11),
        # FIXED west and east sides: the frozen-ghost reads of edge tiles
        (inputs.steady_slope(perturb=0.05), 6),
    ]


@pytest.mark.parametrize("mode,graph", [(swe.BATCH_PERSISTENT, False), (swe.BATCH_PERSISTENT, True),
                                        (swe.BATCH_ROUNDS, False), (swe.BATCH_ROUNDS, True)])
def test_batch_equals_alone_bitwise(mode, graph):
    mix = small_mix()
    tile = 1
    say(f"batch mode={mode} graph={graph}")
    bt = swe.Batch()
    bt.set_mode(mode, graph)
    bt.set_tile(tile)
    idx = [bt.add_scenario(sc, n) for sc, n in mix]
    bt.run()
    for i, (sc, n) in zip(idx, mix):
        got = bt.read(i)
        ref = alone(sc, n, tile)
        assert got[3]["step"] == n
        for a, b in zip(got[:3], ref[:3]):
            assert np.array_equal(a, b), (sc.name, n)
        assert got[3]["t"] == ref[3]["t"]
    bt.close()


def test_batch_in_segments_equals_one_run():
    mix = small_mix()
    full = swe.Batch()
    seg = swe.Batch()
    for sc, n in mix:
        full.add_scenario(sc, n)
        seg.add_scenario(sc, n)
    full.run()
    for _ in range(6):
        seg.run(max_steps=2)
    for i in range(len(mix)):
        a, b = full.read(i), seg.read(i)
        for x, y in zip(a[:3], b[:3]):
            assert np.array_equal(x, y)
    full.close()
    seg.close()


def test_batch_against_checker():
    mix = small_mix()
    bt = swe.Batch()
    idx = [bt.add_scenario(sc, n) for sc, n in mix]
    bt.run()
    for i, (sc, n) in zip(idx, mix):
        g = bt.read(i)
        o = oracle.Oracle.from_scenario(sc)
        o.step(n)
        assert_front_parity(g, o.state(), TOL_SHOCK, f"{sc.name} {n}")
        assert_epilogue_parity(g[3], o.scalars(), sc, sc.name)
    bt.close()


def test_mitigation_ensemble_full_size_truncated():
    # the batched-ensemble workload at its full 1024 x 1024 size, four members
    # of uneven length: batched == alone bitwise; three members after 50
    # steps against the checker
    members = [inputs.mitigation_coast(1024, 1024, 2.0, seed=1000 + s) for s in range(4)]
    steps = [50, 50, 50, 35]
    bt = swe.Batch()
    tile = 1
    bt.set_tile(tile)
    for sc, n in zip(members, steps):
        bt.add_scenario(sc, n)
    bt.run()
    for i, (sc, n) in enumerate(zip(members, steps)):
        g = bt.read(i)
        ref = alone(sc, n, tile)
        for a, b in zip(g[:3], ref[:3]):
            assert np.array_equal(a, b)
        if i < 3:
            o = oracle.Oracle.from_scenario(sc)
            o.step(n)
            assert_front_parity(g, o.state(), TOL_SHOCK, f"ensemble member {i}")
            assert_epilogue_parity(g[3], o.scalars(), sc, f"ensemble member {i}")
    bt.close()


def test_uneven_batch_full_sizes_truncated():
    plan = inputs.uneven_plan()
    picks = []
    for size in inputs.UNEVEN_SIZES:
        s = next(i for i, (sz, _) in enumerate(plan) if sz == size)
        picks.append(s)
    scen = [inputs.uneven_scenario(s, plan) for s in picks]
    steps = [20, 20, 20, 20]
    bt = swe.Batch()
    for sc, n in zip(scen, steps):
        bt.add_scenario(sc, n)
    bt.run()
    for i, (sc, n) in enumerate(zip(scen, steps)):
        g = bt.read(i)
        assert g[3]["step"] == n
        ref = alone(sc, n, 1)  # every tile variant gives the same state
        for a, b in zip(g[:3], ref[:3]):
            assert np.array_equal(a, b), sc.name
    # every size class after 20 steps against the checker
    for i, (sc, n) in enumerate(zip(scen, steps)):
        o = oracle.Oracle.from_scenario(sc)
        assert o.step(n) == 0
        g = bt.read(i)
        assert_front_parity(g, o.state(), TOL_SHOCK, f"uneven {sc.name}")
        assert_epilogue_parity(g[3], o.scalars(), sc, f"uneven {sc.name}")
    bt.close()


def test_nwave_beach_with_hill_against_checker():
    # Carrier N-wave on a 1/10 beach with a coastal hill (Section 2.4), in a
    # batch with a hill-less twin: batched == alone, and against the checker
    sc = inputs.nwave_beach(nx=1024, ny=96, dx=4.0)
    twin = inputs.nwave_beach(nx=1024, ny=96, dx=4.0, hill=False)
    bt = swe.Batch()
    bt.add_scenario(sc, 40)
    bt.add_scenario(twin, 40)
    bt.run()
    g = bt.read(0)
    ref = alone(sc, 40, 4)
    for a, b in zip(g[:3], ref[:3]):
        assert np.array_equal(a, b)
    o = oracle.Oracle.from_scenario(sc)
    o.step(40)
    assert_front_parity(g, o.state(), TOL_SHOCK, "nwave")
    assert_epilogue_parity(g[3], o.scalars(), sc, "nwave")
    bt.close()


@pytest.mark.parametrize("mode,graph", [(swe.BATCH_ROUNDS, True), (swe.BATCH_PERSISTENT, False)])
def test_compensated_batch_equals_compensated_contexts_and_keeps_mass(mode, graph):
    # the compensated level in a batch (SWE_OPT_COMPENSATED): each member
    # advances bitwise as a context with the option, and the mass balance of
    # the shallow 256^2 beach scenario holds to 1e-12 of the mass per step
    plan = inputs.uneven_plan()
    small = next(i for i, (sz, _) in enumerate(plan) if sz == (256, 256))
    mix = [(inputs.uneven_scenario(small, plan), 400), (inputs.random_wet(130, 70, seed=2, dry_fraction=0.05), 9),
           (inputs.parabolic_bowl(nx=150, ny=9, dx=4.0), 31)]
    bt = swe.Batch()
    bt.set_mode(mode, graph)
    bt.set_tile(1)
    bt.add_scenario(*mix[0])
    bt.set_option(swe.OPT_COMPENSATED, 1)  # present members get planes ...
    for sc, n in mix[1:]:
        bt.add_scenario(sc, n)             # ... and members added later too
    m0 = bt.stats(0)["mass"]
    bt.run()
    for i, (sc, n) in enumerate(mix):
        g = bt.read(i)
        s = swe.Solver.from_scenario(sc)
        s.set_option(swe.OPT_TILE, 1)
        s.set_option(swe.OPT_COMPENSATED, 1)
        s.step(n)
        ref = s.read()
        s.close()
        for a, b in zip(g[:3], ref[:3]):
            assert np.array_equal(a, b), sc.name
        if i == 0:
            drift = (g[3]["mass"] - m0 - g[3]["clamp_mass"]) / m0 / n
            say("compensated batch mass drift per step", drift)
            assert abs(drift) <= 1e-12
    bt.set_option(swe.OPT_COMPENSATED, 0)
    bt.close()
