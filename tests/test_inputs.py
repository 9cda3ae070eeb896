"""The seeded generator: digests per seed, workload shapes, and invariants."""
import json
import os

import numpy as np

import analytic as A
from paper_2301_12010_amd import inputs

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_generator_digests_are_pinned():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "mk", os.path.join(GOLD, "make_generator_digests.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    want = json.load(open(os.path.join(GOLD, "generator_sha256.json")))
    got = mk.digests()
    for k, v in got.items():
        assert want[k] == v, k
    plan = [[list(s), n] for s, n in inputs.uneven_plan()[:8]]
    assert plan == want["uneven_plan_first8"]


def test_paper_constants_fixture_matches_generators():
    c = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    sc = inputs.steady_slope()
    assert abs(sc.meta["manning"] - c["slope_manning_n"]["value"]) == 0
    assert abs(sc.meta["slope"] - c["slope_gradient"]["value"]) < 1e-15
    assert sc.meta["depth"] == c["slope_depth_m"]["value"]
    assert inputs.G == c["gravity"]["value"]
    # discharge from Manning's law at the printed constants
    q = A.manning_q(c["slope_depth_m"]["value"], c["slope_gradient"]["value"],
                    c["slope_manning_n"]["value"])
    assert abs(sc.meta["q"] - q) < 1e-12


def test_dry_cells_have_no_momentum_and_depths_are_valid():
    for sc in (inputs.large_coast(128, 128, 5.0), inputs.mitigation_coast(128, 128, 2.0, seed=1001),
               inputs.random_wet(40, 30, seed=1, dry_fraction=0.2), inputs.parabolic_bowl()):
        for a in sc.fields():
            assert a.dtype == np.float32 and np.all(np.isfinite(a))
        assert np.all(sc.h >= 0) and np.all(sc.n >= 0)
        dry = sc.h <= sc.params.h_dry
        assert np.all(sc.hu[dry] == 0) and np.all(sc.hv[dry] == 0)


def test_beach_profile():
    sc = inputs.large_coast(256, 64, 80.0)  # 20.48 km like the 4096 x 5 m grid
    b = sc.b.astype(np.float64)
    # x_s = 0.8 Lx, slope 1/200, clamp [-100, 20]; bumps perturb it by <= 3 m
    assert abs(np.median(b[:, 0]) - (40.0 - 16384.0) / 200.0) < 0.5
    assert np.all(b <= 20.0 + 3.0 + 1e-4)
    sc2 = inputs.mitigation_coast(1024, 64, 2.0, seed=1000)
    assert sc2.meta["xs"] == 0.8 * 2048.0
    assert np.all(sc2.n >= 0.02 - 1e-7) and np.all(sc2.n <= 0.1 + 1e-7)


def test_uneven_plan_shape():
    plan = inputs.uneven_plan()
    assert len(plan) == 200
    assert {s for s, _ in plan} <= set(inputs.UNEVEN_SIZES)
    assert all(1000 <= n <= 4000 for _, n in plan)


def test_nwave_shape_follows_section_2_4():
    import json
    c = json.load(open(os.path.join(GOLD, "paper_constants.json")))["nwave"]
    lam, A = c["lambda"], c["A"]
    x1 = 1000 + c["x1_factor"] * lam
    x2 = 1000 + c["x2_factor"] * lam
    x = np.linspace(0, 6000, 60001)
    eta = inputs.nwave_surface(x, A, lam)
    # crest near x1 of height ~2 a1, trough near x2 of depth ~2 a2: the second
    # exponent decays (read with its minus sign)
    i_max, i_min = np.argmax(eta), np.argmin(eta)
    assert abs(x[i_max] - x1) < 0.05 * lam and abs(eta[i_max] - 2 * A) < 0.05 * 2 * A
    assert abs(x[i_min] - x2) < 0.05 * lam and eta[i_min] < -0.5 * 2 * A * c["a2_over_a1"]
    assert abs(eta[0]) < 1e-3 and abs(eta[-1]) < 1e-3
    sc = inputs.nwave_beach(nx=512, ny=32, dx=8.0)
    assert np.all(sc.h >= 0) and sc.b.max() <= 20 + 8 + 1e-4
