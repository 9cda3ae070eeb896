"""Pins of the FP64 checker against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the checker's
formulas: they compare it with closed forms (Stoker dam break, Thacker bowl,
Manning uniform flow, lake at rest), polynomial exactness of the WENO5
reconstruction, conservation, and exact symmetries of the discrete operator.
"""
import dataclasses

import numpy as np
import pytest

import analytic as A
import oracle
from paper_2301_12010_amd import inputs

F64 = np.float64


def run_to(o, t_end):
    while o.scalars()["t"] < t_end:
        assert o.step(1) == 0
    return o.scalars()


# ---------------------------------------------------------------------------
# WENO5 reconstruction (Methods, WENO paragraph; Jiang & Shu)
# ---------------------------------------------------------------------------

def _fd_derivative(f, x, dx, eps):
    """(fhat_{i+1/2} - fhat_{i-1/2})/dx with fhat = R+(f_{i-2..i+2})."""
    fp = oracle.weno5([f(x + k * dx) for k in (-2, -1, 0, 1, 2)], eps)[0]
    fm = oracle.weno5([f(x + k * dx) for k in (-3, -2, -1, 0, 1)], eps)[0]
    return (fp - fm) / dx


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4, 5])
def test_weno5_linear_weights_exact_to_degree_5(deg):
    # with the linear weights the flux difference is the 6-point upwind
    # derivative, exact for polynomials of degree <= 5
    x, dx = 0.37, 0.1
    f = lambda s: s ** deg
    d = _fd_derivative(f, x, dx, eps=1e30)
    exact = deg * x ** (deg - 1) if deg else 0.0
    assert abs(d - exact) <= 1e-11 * max(1.0, abs(exact))


def test_weno5_linear_weights_not_exact_at_degree_6():
    x, dx = 0.37, 0.1
    d = _fd_derivative(lambda s: s ** 6, x, dx, eps=1e30)
    assert abs(d - 6 * x ** 5) > 1e-6


def test_weno5_fifth_order_with_nonlinear_weights():
    # smooth data, default epsilon: error falls like dx^5
    f = lambda s: np.sin(s)
    errs = [abs(_fd_derivative(f, 0.4, dx, 1e-6) - np.cos(0.4)) for dx in (0.2, 0.1)]
    assert errs[0] / errs[1] > 20.0


def test_weno5_odd_symmetry_bitwise():
    rng = np.random.default_rng(11)
    for _ in range(200):
        v = rng.standard_normal(5) * rng.uniform(1e-3, 1e3)
        r, w = oracle.weno5(v)
        rn, wn = oracle.weno5(-v)
        assert rn == -r
        assert np.array_equal(w, wn)


def test_weno5_weights_on_step_and_normalisation():
    # a jump between v[2] and v[3]: only the left stencil is smooth
    r, w = oracle.weno5([0.0, 0.0, 0.0, 1.0, 1.0])
    assert w[0] > 1 - 1e-10 and w[1] + w[2] < 1e-10
    assert abs(r) < 1e-10
    rng = np.random.default_rng(3)
    for _ in range(100):
        _, w = oracle.weno5(rng.standard_normal(5))
        assert abs(w.sum() - 1.0) <= 4 * np.finfo(float).eps


# ---------------------------------------------------------------------------
# Wet dam break (Section 2.1)
# ---------------------------------------------------------------------------

def test_stoker_closed_form_is_consistent():
    # the quartic's root must satisfy the Rankine-Hugoniot conditions of the
    # right-moving bore with the rarefaction's Riemann invariant
    g, hl, hr = 9.81, 2.0, 1.0
    cm = A.stoker_cm(hl, hr)
    hm = cm * cm / g
    um = 2.0 * (np.sqrt(g * hl) - cm)
    _, _, x3, _ = A.dam_break_fronts(1.0, hl, hr, 0.0)
    s = x3  # shock speed
    assert abs(s * (hm - hr) - hm * um) < 1e-10  # mass
    mom = s * hm * um - (hm * um * um + 0.5 * g * (hm * hm - hr * hr))
    assert abs(mom) < 1e-9  # momentum
    assert np.sqrt(g * hr) < cm < np.sqrt(g * hl)


def test_dam_break_config_against_stoker():
    sc = inputs.dam_break()  # 128 x 64, dx = 1, CFL 0.4, 200 steps, reflective walls
    o = oracle.Oracle.from_scenario(sc)
    assert o.step(sc.nsteps) == 0
    s = o.scalars()
    h, hu, hv = o.state()
    # CFL 0.4 with dt = cfl/(ax/dx + ay/dy): 200 steps end before any wave
    # reaches a wall
    assert 8.0 < s["t"] < 9.0
    x = (np.arange(sc.params.nx) + 0.5) * sc.params.dx
    ha = A.dam_break_h(x, s["t"], 2.0, 1.0, 64.0)
    x1, x2, x3, _ = A.dam_break_fronts(s["t"], 2.0, 1.0, 64.0)
    assert 0 < x1 and x3 < 128
    for row in (0, 31, 63):
        assert A.rel_l2(h[row], ha) < 2.0e-2
        assert A.rel_linf(h[row], ha) < 0.2
        away = (np.abs(x - x1) > 3) & (np.abs(x - x2) > 3) & (np.abs(x - x3) > 3)
        assert A.rel_l2(h[row][away], ha[away]) < 2.5e-3
    # a y-uniform problem stays y-uniform bitwise and hv stays exactly zero
    assert np.array_equal(h, np.broadcast_to(h[0], h.shape))
    assert np.all(hv == 0.0)


def test_dam_break_converges_first_order_in_l1():
    errs = []
    for nx, dx in [(128, 1.0), (256, 0.5), (512, 0.25)]:
        o = oracle.Oracle.from_scenario(inputs.dam_break(nx=nx, ny=3, dx=dx))
        s = run_to(o, 8.0)
        h = o.state()[0][1]
        x = (np.arange(nx) + 0.5) * dx
        errs.append(np.mean(np.abs(h - A.dam_break_h(x, s["t"], 2.0, 1.0, 64.0))))
    assert errs[0] / errs[1] > 1.7 and errs[1] / errs[2] > 1.7


def test_reflective_wall_mass_flux_is_zero():
    # a wave hitting the walls: mass is conserved to rounding of the sum
    sc = inputs.dam_break(nx=40, ny=3, dx=1.0, x0=10.0)
    o = oracle.Oracle.from_scenario(sc)
    m0 = o.scalars()["mass"]
    o.step(800)
    s = o.scalars()
    assert s["t"] > 30.0  # several wall reflections
    assert abs(s["mass"] - m0) <= 1e-13 * m0


# ---------------------------------------------------------------------------
# Planar parabolic bowl (Section 2.2): wet/dry fronts
# ---------------------------------------------------------------------------

def test_parabolic_bowl_converges():
    h0, a, L, amp = 1.0, 200.0, 600.0, 20.0
    T = 2 * np.pi / A.bowl_omega(h0, a)
    errs = []
    for nx, dx in [(300, 2.0), (600, 1.0), (1200, 0.5)]:
        sc = inputs.parabolic_bowl(nx=nx, ny=3, dx=dx, dtype=F64)
        o = oracle.Oracle.from_scenario(sc)
        s = run_to(o, 0.3 * T)
        h, hu, _ = o.state()
        x = (np.arange(nx) + 0.5) * dx
        errs.append(A.rel_l2(h[1], A.bowl_h(x, s["t"], h0, a, L, amp)))
        # velocity in the wet core follows amp * omega * sin(omega t)
        core = A.bowl_h(x, s["t"], h0, a, L, amp) > 0.3
        u = hu[1][core] / h[1][core]
        assert abs(np.median(u) - A.bowl_u(s["t"], h0, a, amp)) < 0.05 * amp * A.bowl_omega(h0, a)
    # the fronts are kinks of h moving over dry land: the error falls with
    # dx, at less than second order (3.2e-3, 2.0e-3, 7.9e-4)
    assert errs[0] < 5e-3
    assert errs[0] / errs[1] > 1.4 and errs[1] / errs[2] > 1.4 and errs[0] / errs[2] > 3.0


def test_mass_balance_with_clamping():
    # |M(t) - M(0) - clamp(t)| / M(0) <= 1e-12, with clamping active
    sc = inputs.parabolic_bowl(nx=300, ny=3, dx=2.0, dtype=F64)
    o = oracle.Oracle.from_scenario(sc)
    m0 = o.scalars()["mass"]
    o.step(300)
    s = o.scalars()
    assert s["clamp_mass"] > 1e-4 * m0  # clamping is active (7.7e-4 of the mass)
    assert abs(s["mass"] - m0 - s["clamp_mass"]) <= 1e-12 * m0


# ---------------------------------------------------------------------------
# Steady flow down a slope with friction (Section 2.3)
# ---------------------------------------------------------------------------

def test_manning_discharge_value():
    # n = 0.033, slope 1/20, depth 0.5 (Section 2.3)
    assert abs(A.manning_q(0.5, 1 / 20, 0.033) - 2.1342947832) < 1e-9


def test_steady_slope_is_discrete_steady_state():
    sc = inputs.steady_slope(dtype=F64)
    o = oracle.Oracle.from_scenario(sc)
    Lh, Lhu, Lhv = o.rhs()
    assert np.abs(Lh).max() < 1e-12
    assert np.abs(Lhu).max() < 1e-12
    assert np.abs(Lhv).max() == 0.0


def test_steady_slope_relaxes_to_manning_flow():
    sc = inputs.steady_slope(perturb=0.05, dtype=F64)
    o = oracle.Oracle.from_scenario(sc)
    q = A.manning_q(0.5, 1 / 20, 0.033)
    run_to(o, 5.0)
    h, hu, _ = o.state()
    assert A.rel_linf(hu, np.full_like(hu, q)) > 1e-3  # still perturbed
    run_to(o, 100.0)
    h, hu, _ = o.state()
    assert A.rel_linf(hu, np.full_like(hu, q)) < 1e-10
    assert A.rel_linf(h, np.full_like(h, 0.5)) < 1e-10


# ---------------------------------------------------------------------------
# Lake at rest (bed source after Xing & Shu, Methods)
# ---------------------------------------------------------------------------

def test_lake_at_rest_preserved_to_roundoff():
    sc = inputs.lake_at_rest(dtype=F64)
    o = oracle.Oracle.from_scenario(sc)
    assert o.step(1000) == 0
    h, hu, hv = o.state()
    assert np.abs(hu).max() <= 1e-10 and np.abs(hv).max() <= 1e-10
    assert np.abs(h + sc.b - 1.7).max() <= 1e-11


def test_steady_slope_on_land_is_an_exact_discrete_steady_state():
    # the same uniform flow with the whole channel above the datum, where the
    # pressure flux is 1/2 g h^2 and the bed source -g h db/dx (reading R2):
    # uniform h and linear b again make L(u) vanish to roundoff
    sc = inputs.steady_slope(b0=5.0, dtype=F64)
    assert sc.b.min() > 1.0
    o = oracle.Oracle.from_scenario(sc)
    assert max(np.abs(a).max() for a in o.rhs()) < 2e-14


def test_lake_at_rest_with_friction_and_anisotropic_cells():
    sc = inputs.lake_at_rest(nx=40, ny=24, dx=1.0, dy=2.5, manning=0.05, dtype=F64)
    o = oracle.Oracle.from_scenario(sc)
    o.step(300)
    h, hu, hv = o.state()
    assert np.abs(hu).max() <= 1e-10 and np.abs(hv).max() <= 1e-10
    assert np.abs(h + sc.b - 1.7).max() <= 1e-11


def test_still_sea_at_the_datum_next_to_dry_land_stays_at_rest():
    # sea at rest at the datum against a beach with hills and a dry curved
    # island (reading R2: the bed relative to the datum).  The state is the
    # exact solution: L(u) vanishes exactly, and over 200 steps the state
    # moves only by the rounding of the RK weights 3/4 and 1/3 (observed
    # 6e-15 m, momentum 4e-14 m^2/s): no water appears on land, the runup
    # stays 0 and nothing of note is clamped.
    sc = inputs.still_coast(dtype=F64)
    o = oracle.Oracle.from_scenario(sc)
    land = sc.b > 0
    assert land.sum() > 0.3 * sc.b.size  # a third of the grid is dry land
    assert all(not a.any() for a in o.rhs())
    m0 = o.scalars()["mass"]
    for _ in range(4):
        assert o.step(50) == 0
        h, hu, hv = o.state()
        assert np.abs(h - sc.h).max() <= 1e-13 and h[land].max() <= 1e-13
        assert np.abs(hu).max() <= 1e-12 and np.abs(hv).max() <= 1e-12
        s = o.scalars()
        assert s["runup"] == 0.0 and s["clamp_mass"] <= 1e-14 * m0
        assert abs(s["mass"] - m0) <= 1e-13 * m0


def test_still_sea_at_the_datum_with_a_wave_keeps_the_land_dry_ahead_of_it():
    # the same coast with a wave far offshore: until the wave arrives the
    # land ahead of it stays dry and the momentum there stays zero
    sc = inputs.still_coast(dtype=F64)
    X = (np.arange(sc.params.nx) + 0.5) * sc.params.dx
    hump = 0.2 * np.exp(-((X - 10.0) / 5.0) ** 2)
    h = np.where(sc.b < 0, np.maximum(hump - sc.b, 0.0), 0.0)
    o = oracle.Oracle(sc.params, sc.b, sc.n, h, sc.hu, sc.hv)
    assert o.step(10) == 0
    h1, hu1, _ = o.state()
    far = X > 0.5 * sc.params.nx * sc.params.dx  # beyond the island
    assert np.abs(h1[:, far] - h[:, far]).max() <= 1e-13
    assert np.abs(hu1[:, far]).max() <= 1e-12
    assert o.scalars()["runup"] == 0.0


# ---------------------------------------------------------------------------
# TVD-RK3 (Methods, Eq. (8)): third order in time
# ---------------------------------------------------------------------------

def test_rk3_third_order_in_time():
    nx = 80
    x = (np.arange(nx) + 0.5)
    h = 1.0 + 0.1 * np.exp(-((x - 40.0) / 6.0) ** 2)
    z = np.zeros((3, nx))
    H = np.broadcast_to(h, (3, nx)).copy()

    def run(dt, T=4.0):
        p = inputs.Params(nx, 3, 1.0, 1.0, cfl=0.0, dt_fixed=dt)
        o = oracle.Oracle(p, z, z, H, z, z)
        o.step(int(round(T / dt)))
        return o.state()[0][1]

    ref = run(0.00625)
    e = [np.abs(run(dt) - ref).max() for dt in (0.2, 0.1, 0.05)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 6.0 < r1 < 10.0 and 6.0 < r2 < 10.0


# ---------------------------------------------------------------------------
# Exact symmetries of the discrete operator
# ---------------------------------------------------------------------------

def _run(sc, n):
    o = oracle.Oracle.from_scenario(sc)
    assert o.step(n) == 0
    return o.state(), o.scalars()


def test_transpose_symmetry_bitwise():
    sc = inputs.random_wet(37, 23, seed=4, dry_fraction=0.05)
    (h, hu, hv), s = _run(sc, 12)
    (hT, huT, hvT), sT = _run(inputs.transpose(sc), 12)
    assert np.array_equal(hT, h.T) and np.array_equal(huT, hv.T) and np.array_equal(hvT, hu.T)
    assert s["t"] == sT["t"]


def test_mirror_symmetry_bitwise():
    sc = inputs.random_wet(33, 17, seed=9, dry_fraction=0.05)
    (h, hu, hv), _ = _run(sc, 12)
    (hM, huM, hvM), _ = _run(inputs.mirror_x(sc), 12)
    assert np.array_equal(hM, h[:, ::-1])
    assert np.array_equal(huM, -hu[:, ::-1])
    assert np.array_equal(hvM, hv[:, ::-1])


def test_runup_is_non_decreasing():
    sc = inputs.parabolic_bowl(nx=300, ny=3, dx=2.0)
    o = oracle.Oracle.from_scenario(sc)
    r = [o.scalars()["runup"]]
    for _ in range(10):
        o.step(40)
        r.append(o.scalars()["runup"])
    assert all(b >= a for a, b in zip(r, r[1:]))


def test_invalid_inputs_rejected():
    sc = inputs.dam_break(nx=8, ny=4)
    bad = sc.h.copy()
    bad[1, 1] = np.nan
    with pytest.raises(ValueError):
        oracle.Oracle(sc.params, sc.b, sc.n, bad, sc.hu, sc.hv)
    bad = sc.h.copy()
    bad[0, 0] = -1.0
    with pytest.raises(ValueError):
        oracle.Oracle(sc.params, sc.b, sc.n, bad, sc.hu, sc.hv)
    small = inputs.dam_break(nx=2, ny=4)
    with pytest.raises(ValueError):
        oracle.Oracle.from_scenario(small)


# ---------------------------------------------------------------------------
# Point-implicit friction, the variant the paper declines (Methods; reading
# R10 of the checker)
# ---------------------------------------------------------------------------

def decay_errors(L=None, dts=(0.25, 0.125, 0.0625), T=2.0):
    """Relative error of the mid-channel discharge at time T against the
    friction decay law, per time step; also checks h and the sign of q."""
    errs = []
    for dt in dts:
        sc = inputs.friction_channel(dt_fixed=dt, dtype=F64)
        o = oracle.Oracle.from_scenario(sc, L=L)
        o.set_friction(True)
        qs = []
        for _ in range(int(round(T / dt))):
            assert o.step(1) == 0
            h, hu, hv = o.state()
            qs.append(hu[1, sc.params.nx // 2])
            assert h[1, sc.params.nx // 2] == sc.meta["depth"]
        qs = np.array(qs)
        assert np.all(qs > 0) and np.all(np.diff(qs) <= 0)
        exact = A.friction_decay_q(T, sc.meta["q0"], sc.meta["depth"], sc.meta["manning"])
        errs.append(abs(qs[-1] - exact) / exact)
    return errs


def test_implicit_friction_converges_to_the_decay_law():
    # kappa dt = 1.3 to 0.33 at the start: first order in dt (each stage
    # takes its friction backward in time with the rate of its input)
    errs = decay_errors()
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2
    assert errs[2] < 0.035


def test_implicit_friction_is_stable_where_explicit_is_not():
    # Manning n = 10 on a 5 cm film: kappa dt ~ 2.7e3 at the start
    sc = inputs.friction_channel(manning=10.0, dt_fixed=0.5, dtype=F64)
    mid = sc.params.nx // 2
    o = oracle.Oracle.from_scenario(sc)
    o.set_friction(True)
    qs = []
    for _ in range(8):
        assert o.step(1) == 0
        qs.append(o.state()[1][1, mid])
    assert np.all(np.diff([sc.meta["q0"]] + qs) < 0) and min(qs) > 0
    e = oracle.Oracle.from_scenario(sc)  # explicit, no stiffness cap
    rc = e.step(3)
    q = e.state()[1][1, mid]
    assert rc != 0 or not np.isfinite(q) or q < 0 or q > sc.meta["q0"]


def test_implicit_friction_keeps_the_steady_slope():
    # the Manning discharge balances the bed slope; taking the friction
    # implicitly leaves that exact discrete steady state in place
    sc = inputs.steady_slope(dtype=F64)
    o = oracle.Oracle.from_scenario(sc)
    o.set_friction(True)
    o.step(50)
    h, hu, hv = o.state()
    assert np.abs(h - sc.h).max() < 1e-12
    assert np.abs(hu - sc.hu).max() < 1e-11
    assert np.abs(hv).max() == 0.0


def test_friction_cap_cuts_a_stiff_rate_to_one_over_dt():
    # Manning n = 10 on a 5 cm film with kappa_cap = 1 (reading R8): kappa dt
    # is ~2.7e4 at the start, above the cap 1/dt at every stage that sees
    # flow.  Mid-channel only friction acts, so stage 1 removes the whole
    # discharge (q1 = q - dt (1/dt) q = 0), stage 2 sees no flow and keeps
    # 3/4 q^n, stage 3 removes its input's discharge again and ends at
    # (1/3) q^n: the discharge falls by exactly a factor 3 per step while
    # the depth stays.
    sc = inputs.friction_channel(manning=10.0, dt_fixed=0.5, kappa_cap=1.0, dtype=F64)
    mid = sc.params.nx // 2
    o = oracle.Oracle.from_scenario(sc)
    (h1, hu1, _), dt = o.stage1()
    assert dt == 0.5 and hu1[1, mid] == 0.0 and h1[1, mid] == sc.meta["depth"]
    q = sc.meta["q0"]
    for _ in range(6):
        assert o.step(1) == 0
        h, hu, hv = o.state()
        q = q / 3.0
        assert abs(hu[1, mid] - q) <= 1e-14 * q
        assert h[1, mid] == sc.meta["depth"] and hv[1, mid] == 0.0


def test_implicit_friction_without_manning_is_the_explicit_scheme():
    sc = inputs.random_wet(24, 18, seed=4, dry_fraction=0.1, manning=0.0)
    a = oracle.Oracle.from_scenario(sc)
    b = oracle.Oracle.from_scenario(sc)
    b.set_friction(True)
    a.step(6)
    b.step(6)
    for x, y in zip(a.state(), b.state()):
        assert np.array_equal(x, y)


# ---------------------------------------------------------------------------
# Time step and runup diagnostics (Methods, Eq. (7) and the Lax-Friedrichs
# paragraph: global wave speeds; Section 2.4: runup)
# ---------------------------------------------------------------------------

def dt_of_first_step(params, fields):
    o = oracle.Oracle(params, *fields)
    assert o.step(1) == 0
    return o.scalars()["dt"]


def test_time_step_of_still_water_is_the_gravity_wave_limit():
    # still water: the fastest signal in either direction is the gravity
    # wave sqrt(g h) of the deepest cell
    sc = inputs.lake_at_rest(nx=32, ny=28, dx=1.0, dy=2.0, dtype=F64)
    c = np.sqrt(9.81 * sc.h.max())
    expect = sc.params.cfl / (c / 1.0 + c / 2.0)
    assert abs(dt_of_first_step(sc.params, sc.fields()) - expect) <= 1e-14 * expect


def test_time_step_of_uniform_flow_adds_the_flow_speed_along_x():
    # uniform flow u along x on anisotropic cells: alpha_x = u + sqrt(g h),
    # alpha_y = sqrt(g h)
    sc = inputs.friction_channel(nx=64, dtype=F64)
    p = dataclasses.replace(sc.params, cfl=0.4, dt_fixed=0.0, dx=10.0, dy=25.0)
    u = sc.meta["q0"] / sc.meta["depth"]
    c = np.sqrt(9.81 * sc.meta["depth"])
    expect = 0.4 / ((u + c) / 10.0 + c / 25.0)
    assert abs(dt_of_first_step(p, sc.fields()) - expect) <= 1e-14 * expect


def test_runup_is_the_highest_wet_bed_reached():
    # a lake against a planar beach with a wave offshore: the runup is the
    # highest bed above the datum under water deeper than h_dry, over the
    # starting state and the state after every step (brute force over that
    # definition on a small grid)
    nx, ny, dx = 60, 5, 1.0
    X = (np.arange(nx) + 0.5) * dx
    b = np.tile(0.05 * (X - 30.0), (ny, 1))
    h = np.maximum(0.3 + 0.4 * np.exp(-((X - 12.0) / 4.0) ** 2) - b, 0.0)
    z = np.zeros_like(b)
    p = inputs.Params(nx, ny, dx, dx, cfl=0.4)
    o = oracle.Oracle(p, b, z, h, z, z)

    def highest_wet_bed(depth):
        m = (b > 0) & (depth > p.h_dry)
        return b[m].max() if m.any() else 0.0

    best = highest_wet_bed(h)
    assert o.scalars()["runup"] == best
    for _ in range(120):
        assert o.step(1) == 0
        best = max(best, highest_wet_bed(o.state()[0]))
        assert o.scalars()["runup"] == best
    assert best > highest_wet_bed(h)  # the wave climbed the beach


# ---------------------------------------------------------------------------
# Local Lax-Friedrichs splitting, the variant of the Methods' global speed
# (reading R11 of the checker: each face splits the six cells its two
# reconstructions read with the largest normal speed among them)
# ---------------------------------------------------------------------------

def fastest_every_third_cell():
    """A y-uniform state whose x speed peaks at every third cell: every
    face's six-cell stencil (ghosts included) holds the fastest cell."""
    nx, ny = 60, 5
    i = np.arange(nx)
    hu = np.tile(np.where(i % 3 == 0, 0.5, 0.1), (ny, 1))
    z = np.zeros((ny, nx))
    return inputs.Params(nx, ny, 1.0, 1.0, cfl=0.4), np.full((ny, nx), -2.0), z, np.ones((ny, nx)), hu, z


def test_local_lf_is_the_global_split_where_every_stencil_holds_the_fastest_cell():
    a = oracle.Oracle(*fastest_every_third_cell())
    b = oracle.Oracle(*fastest_every_third_cell())
    b.set_split(True)
    (ga, dta), (gb, dtb) = a.stage1(), b.stage1()
    assert dta == dtb
    assert all(np.array_equal(x, y) for x, y in zip(ga, gb))
    assert np.abs(ga[1] - fastest_every_third_cell()[4]).max() > 1e-3  # the stage did change hu


def test_local_lf_keeps_still_water_at_rest():
    sc = inputs.lake_at_rest(dtype=F64)
    o = oracle.Oracle.from_scenario(sc)
    o.set_split(True)
    assert o.step(1000) == 0
    h, hu, hv = o.state()
    assert np.abs(hu).max() <= 1e-10 and np.abs(hv).max() <= 1e-10
    assert np.abs(h + sc.b - 1.7).max() <= 1e-11
    sc = inputs.still_coast(dtype=F64)
    o = oracle.Oracle.from_scenario(sc)
    o.set_split(True)
    assert o.step(200) == 0
    h, hu, _ = o.state()
    assert np.abs(h - sc.h).max() <= 1e-13 and np.abs(hu).max() <= 1e-12
    assert o.scalars()["runup"] == 0.0


def test_local_lf_dam_break_against_stoker():
    sc = inputs.dam_break()
    o = oracle.Oracle.from_scenario(sc)
    o.set_split(True)
    assert o.step(sc.nsteps) == 0
    s = o.scalars()
    h = o.state()[0]
    x = (np.arange(sc.params.nx) + 0.5) * sc.params.dx
    ha = A.dam_break_h(x, s["t"], 2.0, 1.0, 64.0)
    x1, x2, x3, _ = A.dam_break_fronts(s["t"], 2.0, 1.0, 64.0)
    away = (np.abs(x - x1) > 3) & (np.abs(x - x2) > 3) & (np.abs(x - x3) > 3)
    assert A.rel_l2(h[31], ha) < 2.0e-2 and A.rel_l2(h[31][away], ha[away]) < 2.5e-3
    assert np.array_equal(h, np.broadcast_to(h[0], h.shape))


def test_local_lf_bowl_fronts_are_less_diffused():
    # small speeds near the wet/dry fronts give a smaller local viscosity:
    # the bowl's error falls 4x against the global speed (2.0e-3 -> 5.3e-4 at
    # dx = 1) and still falls with dx
    h0, a, L, amp = 1.0, 200.0, 600.0, 20.0
    T = 2 * np.pi / A.bowl_omega(h0, a)
    errs = {}
    for local in (False, True):
        for nx, dx in [(300, 2.0), (600, 1.0)]:
            sc = inputs.parabolic_bowl(nx=nx, ny=3, dx=dx, dtype=F64)
            o = oracle.Oracle.from_scenario(sc)
            o.set_split(local)
            s = run_to(o, 0.3 * T)
            x = (np.arange(nx) + 0.5) * dx
            errs[local, dx] = A.rel_l2(o.state()[0][1], A.bowl_h(x, s["t"], h0, a, L, amp))
            m0 = float(np.sum(sc.h)) * dx * dx
            assert abs(s["mass"] - m0 - s["clamp_mass"]) <= 1e-12 * m0
    assert errs[True, 1.0] < 0.5 * errs[False, 1.0]
    assert errs[True, 1.0] < errs[True, 2.0]


def test_local_lf_symmetries_and_walls():
    sc = inputs.random_wet(33, 17, seed=9, dry_fraction=0.05)
    runs = []
    for s_ in (sc, inputs.mirror_x(sc), inputs.transpose(sc)):
        o = oracle.Oracle.from_scenario(s_)
        o.set_split(True)
        assert o.step(12) == 0
        runs.append(o.state())
    (h, hu, hv), (hM, huM, hvM), (hT, huT, hvT) = runs
    assert np.array_equal(hM, h[:, ::-1]) and np.array_equal(huM, -hu[:, ::-1])
    assert np.array_equal(hT, h.T) and np.array_equal(huT, hv.T) and np.array_equal(hvT, hu.T)
    o = oracle.Oracle.from_scenario(inputs.dam_break(nx=40, ny=3, x0=10.0))
    o.set_split(True)
    m0 = o.scalars()["mass"]
    o.step(800)
    assert abs(o.scalars()["mass"] - m0) <= 1e-13 * m0
