"""Seeded synthetic inputs for the shallow-water step.

This module builds bathymetry, Manning-n and initial-state fields.  It holds
none of the solver's arithmetic (no fluxes, no reconstruction, no time
stepping), so both the HIP library and the FP64 reference checker may be fed
from it.  Every field is generated in float64 from a NumPy ``PCG64`` stream
and rounded once to float32; those float32 values are what every solver sees.

Workloads follow the paper's verification and validation problems:

* planar wet dam break (Stoker), Section 2.1;
* planar parabolic bowl (Thacker), Section 2.2;
* steady flow down a slope with Manning friction, Section 2.3;
* lake at rest over a submerged, smooth random bed (well-balance check of the
  bed source term the Methods section takes from Xing & Shu);
* synthetic coastlines standing in for the paper's beach/hill and Crescent
  City runs (Sections 2.4-2.5): a linear beach, Gaussian bumps and hills,
  Manning-n patches, and a Gaussian free-surface hump (the large coastline)
  or Carrier's N-wave (the mitigation ensemble and the uneven batch).

Arrays are row-major ``[ny][nx]`` with x fastest; cell centres sit at
``x_i = (i + 1/2) dx``, ``y_j = (j + 1/2) dy``.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field, replace

import numpy as np

G = 9.81

BC_REFLECT = 0
BC_FIXED = 1


@dataclass
class Params:
    """Scalar problem parameters (mirrors the C ``swe_params`` struct)."""

    nx: int
    ny: int
    dx: float
    dy: float
    g: float = G
    cfl: float = 0.4
    dt_fixed: float = 0.0
    h_dry: float = 1e-3
    weno_eps: float = 1e-6
    kappa_cap: float = 0.0
    bc: tuple = (BC_REFLECT, BC_REFLECT, BC_REFLECT, BC_REFLECT)  # W, E, S, N


@dataclass
class Scenario:
    """One problem: parameters, float32 fields and a step budget."""

    name: str
    params: Params
    b: np.ndarray
    n: np.ndarray
    h: np.ndarray
    hu: np.ndarray
    hv: np.ndarray
    nsteps: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return self.params.nx * self.params.ny

    def fields(self):
        return self.b, self.n, self.h, self.hu, self.hv

    def digest(self) -> str:
        """SHA-256 over the float32 fields (pins the generator per seed)."""
        m = hashlib.sha256()
        for a in self.fields():
            m.update(np.ascontiguousarray(a, dtype=np.float32).tobytes())
        return m.hexdigest()


def _f32(a, dtype=np.float32) -> np.ndarray:
    """Round a float64 field once to ``dtype`` (float32 unless a float64
    verification input is asked for)."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(dtype))


def _centres(nx: int, ny: int, dx: float, dy: float):
    x = (np.arange(nx, dtype=np.float64) + 0.5) * dx
    y = (np.arange(ny, dtype=np.float64) + 0.5) * dy
    return np.meshgrid(x, y)  # X[j, i], Y[j, i]


def _wet_state(eta: np.ndarray, b: np.ndarray, h_dry: float):
    """Water depth from a surface; momentum zero (also on dry cells)."""
    h = np.maximum(eta - b, 0.0)
    z = np.zeros_like(h)
    return h, z, z.copy()


# ---------------------------------------------------------------------------
# Verification problems (paper, Section 2)
# ---------------------------------------------------------------------------

def dam_break(nx: int = 128, ny: int = 64, dx: float = 1.0, h_l: float = 2.0,
              h_r: float = 1.0, x0: float | None = None, cfl: float = 0.4,
              nsteps: int = 200, bc: int = BC_REFLECT, dtype=np.float32) -> Scenario:
    """Planar wet dam break on a flat, frictionless bed (Section 2.1).

    ``h = h_l`` for cell centres left of ``x0`` and ``h_r`` otherwise; with the
    default ``x0 = nx dx / 2`` the dam sits on a cell face.
    """
    if x0 is None:
        x0 = 0.5 * nx * dx
    X, _ = _centres(nx, ny, dx, dx)
    h = np.where(X < x0, h_l, h_r)
    z = np.zeros((ny, nx))
    p = Params(nx, ny, dx, dx, cfl=cfl, bc=(bc, bc, BC_REFLECT, BC_REFLECT))
    f = lambda a: _f32(a, dtype)
    return Scenario("dam_break", p, f(z), f(z), f(h), f(z), f(z),
                    nsteps, dict(h_l=h_l, h_r=h_r, x0=x0))


def parabolic_bowl(nx: int = 600, ny: int = 8, dx: float = 1.0, h0: float = 1.0,
                   a: float = 200.0, amp: float = 20.0, cfl: float = 0.4,
                   nsteps: int = 0, dtype=np.float32) -> Scenario:
    """Planar parabolic bowl (Thacker), Section 2.2, at t = 0.

    Bed ``b = h0((x - L/2)^2/a^2 - 1)`` with ``L = nx dx``; the water surface is
    the bowl's analytic free surface with x-amplitude ``amp`` at t = 0
    (the paper's printed case fixes the amplitude to half a metre).
    """
    L = nx * dx
    X, _ = _centres(nx, ny, dx, dx)
    b = h0 * ((X - 0.5 * L) ** 2 / a ** 2 - 1.0)
    h = -h0 * (((X - 0.5 * L + amp) / a) ** 2 - 1.0)
    h = np.maximum(h, 0.0)
    z = np.zeros((ny, nx))
    # the walls stay dry throughout: mirror ghosts are adequate
    p = Params(nx, ny, dx, dx, cfl=cfl)
    f = lambda a_: _f32(a_, dtype)
    return Scenario("parabolic_bowl", p, f(b), f(z), f(h), f(z), f(z),
                    nsteps, dict(h0=h0, a=a, L=L, amp=amp))


def steady_slope(nx: int = 64, ny: int = 4, dx: float = 1.0, depth: float = 0.5,
                 slope: float = 1.0 / 20.0, manning: float = 0.033,
                 perturb: float = 0.0, cfl: float = 0.4, b0: float = -1.0,
                 dtype=np.float32) -> Scenario:
    """Uniform friction-limited flow down a constant slope (Section 2.3).

    The bed falls along +x with gradient ``slope`` from ``b0`` at the west
    face.  The default puts the bed and its linearly extended ghosts below
    the datum (where the pressure flux is the paper's 1/2 g (h^2 - b^2)); a
    ``b0`` high enough puts the whole channel on land above it (flux
    1/2 g h^2, bed source -g h db/dx).  The uniform unit discharge of
    Manning's law is
    ``q = sqrt(slope)/n * depth^(5/3)``.  West and east sides use frozen
    (FIXED) ghosts, north and south mirror ghosts.  A non-zero ``perturb``
    adds a Gaussian depth bump of relative height ``perturb`` and radius L/10
    at mid-channel (it is below 1e-10 at the ends, so the frozen inflow
    ghosts keep the uniform state).
    """
    X, Y = _centres(nx, ny, dx, dx)
    b = b0 - slope * X
    q = np.sqrt(slope) / manning * depth ** (5.0 / 3.0)
    h = np.full((ny, nx), depth)
    if perturb:
        Lx = nx * dx
        h = h * (1.0 + perturb * np.exp(-((X - 0.5 * Lx) / (0.1 * Lx)) ** 2))
    hu = np.full((ny, nx), q)
    z = np.zeros((ny, nx))
    p = Params(nx, ny, dx, dx, cfl=cfl,
               bc=(BC_FIXED, BC_FIXED, BC_REFLECT, BC_REFLECT))
    f = lambda a: _f32(a, dtype)
    return Scenario("steady_slope", p, f(b), f(np.full((ny, nx), manning)),
                    f(h), f(hu), f(z), 0, dict(q=q, depth=depth, slope=slope,
                                               manning=manning))


def still_coast(nx: int = 64, ny: int = 48, dx: float = 2.0, seed: int = 11,
                manning: float = 0.025, kappa_cap: float = 1.0, dtype=np.float32) -> Scenario:
    """Sea at rest at the datum against a beach with hills and a dry island.

    The beach rises along +x (1/20) through the datum at 0.6 Lx; a Gaussian
    island (4 m high, radius 10 m) stands in the sea at 0.3 Lx with its top
    above the datum, and 2-4 seeded Gaussian hills (3-6 m, radius 6-14 m)
    stand on the land.  Every cell below the datum holds water up to it and
    every cell above it is dry: the exact solution is the initial state.
    Reflective walls.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = _centres(nx, ny, dx, dx)
    Lx, Ly = nx * dx, ny * dx
    b = 0.05 * (X - 0.6 * Lx) + _gauss(X, Y, 4.0, 10.0, 0.3 * Lx, 0.5 * Ly)
    for _ in range(int(rng.integers(2, 5))):
        b = b + _gauss(X, Y, rng.uniform(3.0, 6.0), rng.uniform(6.0, 14.0),
                       rng.uniform(0.7 * Lx, 0.95 * Lx), rng.uniform(0.0, Ly))
    b = _f32(b, dtype)
    h = _f32(np.maximum(-b.astype(np.float64), 0.0), dtype)
    z = np.zeros((ny, nx))
    p = Params(nx, ny, dx, dx, cfl=0.4, kappa_cap=kappa_cap)
    return Scenario("still_coast", p, b, _f32(np.full((ny, nx), manning), dtype), h,
                    _f32(z, dtype), _f32(z, dtype), 0, dict(seed=seed))


def friction_channel(nx: int = 801, ny: int = 3, dx: float = 10.0, depth: float = 0.05,
                     q0: float = 0.05, manning: float = 0.1, dt_fixed: float = 0.25,
                     kappa_cap: float = 0.0, dtype=np.float32) -> Scenario:
    """Uniform flow along x over a flat bed, slowed by Manning friction only.

    West and east sides are frozen (FIXED) ghosts at the initial state, north
    and south mirror ghosts; a fixed time step.  Away from the ends the flux
    gradient vanishes, so the discharge follows the friction decay law.
    """
    z = np.zeros((ny, nx))
    p = Params(nx, ny, dx, dx, cfl=0.0, dt_fixed=dt_fixed, kappa_cap=kappa_cap,
               bc=(BC_FIXED, BC_FIXED, BC_REFLECT, BC_REFLECT))
    f = lambda a: _f32(a, dtype)
    return Scenario("friction_channel", p, f(z), f(np.full((ny, nx), manning)),
                    f(np.full((ny, nx), depth)), f(np.full((ny, nx), q0)), f(z), 0,
                    dict(depth=depth, q0=q0, manning=manning))


def lake_at_rest(nx: int = 48, ny: int = 40, dx: float = 1.0, dy: float | None = None,
                 eta0: float = 1.7, seed: int = 7, nbumps: int = 6,
                 depth: float = 3.0, manning: float = 0.0, cfl: float = 0.4,
                 dtype=np.float32) -> Scenario:
    """Still water with a flat surface ``eta0`` over a smooth random bed.

    The bed is ``eta0 - depth`` plus ``nbumps`` Gaussian bumps, capped a tenth
    of ``depth`` below both the surface and the datum: every cell is
    submerged and the bed lies below the datum, so the exact solution is the
    initial state and the scheme keeps it exactly (``eta0`` is away from the
    datum, so the pressure flux and the bed source do not vanish separately).
    """
    dy = dx if dy is None else dy
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = _centres(nx, ny, dx, dy)
    Lx, Ly = nx * dx, ny * dy
    b = np.full((ny, nx), eta0 - depth)
    for _ in range(nbumps):
        A = rng.uniform(-0.4, 0.6) * depth
        R = rng.uniform(0.08, 0.25) * min(Lx, Ly)
        cx, cy = rng.uniform(0, Lx), rng.uniform(0, Ly)
        b += A * np.exp(-(((X - cx) ** 2 + (Y - cy) ** 2) / R ** 2))
    b = np.minimum(b, min(eta0, 0.0) - 0.1 * depth)
    b = _f32(b, dtype)
    h = _f32(eta0 - b.astype(np.float64), dtype)
    z = np.zeros((ny, nx))
    p = Params(nx, ny, dx, dy, cfl=cfl)
    return Scenario("lake_at_rest", p, b, _f32(np.full((ny, nx), manning), dtype),
                    h, _f32(z, dtype), _f32(z, dtype), 0, dict(eta0=eta0))


def random_wet(nx: int, ny: int, seed: int, dx: float = 1.0, dy: float | None = None,
               dry_fraction: float = 0.0, manning: float = 0.03,
               kappa_cap: float = 1.0) -> Scenario:
    """Random smooth-ish wet state with momentum, for one-stage parity checks.

    With ``dry_fraction > 0`` a seeded set of cells is set to depths around the
    wet/dry threshold and their momentum zeroed.
    """
    dy = dx if dy is None else dy
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = _centres(nx, ny, dx, dy)
    Lx, Ly = nx * dx, ny * dy
    b = -1.0 + 0.3 * np.sin(2 * np.pi * X / Lx * rng.uniform(0.5, 2)) \
        * np.cos(2 * np.pi * Y / Ly * rng.uniform(0.5, 2))
    b += 0.05 * rng.standard_normal((ny, nx))
    h = 1.2 + 0.2 * rng.standard_normal((ny, nx)) - b - 1.0
    h = np.maximum(h, 0.2)
    hu = 0.3 * rng.standard_normal((ny, nx)) * h
    hv = 0.3 * rng.standard_normal((ny, nx)) * h
    n = manning * (1.0 + 0.5 * rng.uniform(size=(ny, nx)))
    if dry_fraction > 0:
        mask = rng.uniform(size=(ny, nx)) < dry_fraction
        h = np.where(mask, rng.uniform(0, 3e-3, size=(ny, nx)), h)
        small = h <= 1e-3
        hu = np.where(small, 0.0, hu)
        hv = np.where(small, 0.0, hv)
    p = Params(nx, ny, dx, dy, cfl=0.4, kappa_cap=kappa_cap)
    return Scenario(f"random_wet_{seed}", p, _f32(b), _f32(n), _f32(h), _f32(hu),
                    _f32(hv), 0, dict(seed=seed))


# ---------------------------------------------------------------------------
# Synthetic coastlines (stand-ins for the paper's beach, hill and DEM runs)
# ---------------------------------------------------------------------------

def _gauss(X, Y, A, R, cx, cy):
    return A * np.exp(-(((X - cx) ** 2 + (Y - cy) ** 2) / R ** 2))


def _beach(X, Lx):
    """Linear beach, slope 1/200, shoreline at 0.8 Lx, clamped to [-100, 20] m."""
    xs = 0.8 * Lx
    return np.clip((X - xs) / 200.0, -100.0, 20.0), xs


def large_coast(nx: int = 4096, ny: int = 4096, dx: float = 5.0, seed: int = 2,
                nsteps: int = 2000, nbumps: int = 32) -> Scenario:
    """Single large coastline: beach + seeded bumps + plane Gaussian hump.

    Bumps: amplitude U(-3, 3) m, width W ~ U(50, 300) m (radius W/2), centres
    uniform in the domain.  Hump: 2 m high, 2 km wide (radius 1 km) centred
    1 km from the offshore edge.  n = 0.025, h_dry = 1e-3, kappa cap on.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = _centres(nx, ny, dx, dx)
    Lx, Ly = nx * dx, ny * dx
    b, xs = _beach(X, Lx)
    for _ in range(nbumps):
        A = rng.uniform(-3.0, 3.0)
        W = rng.uniform(50.0, 300.0)
        cx, cy = rng.uniform(0, Lx), rng.uniform(0, Ly)
        b = b + _gauss(X, Y, A, 0.5 * W, cx, cy)
    eta = 2.0 * np.exp(-((X - 1000.0) / 1000.0) ** 2)
    h, hu, hv = _wet_state(eta, b, 1e-3)
    n = np.full((ny, nx), 0.025)
    p = Params(nx, ny, dx, dx, cfl=0.4, h_dry=1e-3, kappa_cap=1.0)
    return Scenario(f"large_coast_{nx}x{ny}", p, _f32(b), _f32(n), _f32(h), _f32(hu),
                    _f32(hv), nsteps, dict(seed=seed, xs=xs))


def deep_ocean(nx: int = 96, ny: int = 64, dx: float = 1000.0, seed: int = 5,
               depth: float = 4000.0, nseamounts: int = 6) -> Scenario:
    """Open-ocean propagation: a 4 km deep basin with seeded seamounts and
    trenches (amplitude U(-800, 800) m, radius U(5, 15) km) and a 1 m
    Gaussian hump of 8 km radius.  Fully wet and smooth; in FP32 an ocean
    depth has an ulp of 2.4e-4 m, so this case shows whether the stored
    state resolves a metre-scale wave on top of it."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = _centres(nx, ny, dx, dx)
    Lx, Ly = nx * dx, ny * dx
    b = np.full((ny, nx), -depth)
    for _ in range(nseamounts):
        b = b + _gauss(X, Y, rng.uniform(-800.0, 800.0), rng.uniform(5e3, 15e3),
                       rng.uniform(0, Lx), rng.uniform(0, Ly))
    eta = _gauss(X, Y, 1.0, 8e3, 0.3125 * Lx, 0.5 * Ly)
    h, hu, hv = _wet_state(eta, b, 1e-3)
    n = np.full((ny, nx), 0.025)
    p = Params(nx, ny, dx, dx, cfl=0.4, h_dry=1e-3, kappa_cap=1.0)
    return Scenario(f"deep_ocean_{nx}x{ny}", p, _f32(b), _f32(n), _f32(h), _f32(hu),
                    _f32(hv), 0, dict(seed=seed, depth=depth))


def mitigation_coast(nx: int = 1024, ny: int = 1024, dx: float = 2.0, seed: int = 1000,
                     nsteps: int = 3000) -> Scenario:
    """One mitigation-ensemble member: Carrier's N-wave running up a beach
    with coastal hills and Manning patches (the hill-on-a-beach study of
    Section 2.4 as a mitigation ensemble).

    Beach as ``_beach`` (shoreline xs = 0.8 Lx, slope 1/200); 1-8 hills of
    height U(3, 10) m and radius U(20, 80) m centred at x ~ U(xs - 50,
    xs + 150), y ~ U(0, Ly); background n = 0.025 with 1-4 disks of radius
    U(50, 200) m and n ~ U(0.02, 0.1) (later disks win), disk centres
    x ~ U(xs - 200, Lx), y ~ U(0, Ly).  The initial surface is the N-wave of
    ``nwave_surface`` scaled to the grid: A = 1 m (a 2 m crest and a 0.67 m
    leading trough), lambda = 0.2 Lx and the origin 0.05 Lx offshore, so on
    a 1024 x 1024 grid of 2 m cells the crest stands 313 m offshore; water
    at rest, free-slip walls.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = _centres(nx, ny, dx, dx)
    Lx, Ly = nx * dx, ny * dx
    b, xs = _beach(X, Lx)
    for _ in range(int(rng.integers(1, 9))):
        A = rng.uniform(3.0, 10.0)
        R = rng.uniform(20.0, 80.0)
        cx, cy = rng.uniform(xs - 50.0, xs + 150.0), rng.uniform(0, Ly)
        b = b + _gauss(X, Y, A, R, cx, cy)
    n = np.full((ny, nx), 0.025)
    for _ in range(int(rng.integers(1, 5))):
        R = rng.uniform(50.0, 200.0)
        cx, cy = rng.uniform(xs - 200.0, Lx), rng.uniform(0, Ly)
        nv = rng.uniform(0.02, 0.1)
        n = np.where((X - cx) ** 2 + (Y - cy) ** 2 <= R * R, nv, n)
    eta = nwave_surface(xs - X, A=1.0, lam=0.2 * Lx, origin=0.05 * Lx)
    h, hu, hv = _wet_state(eta, b, 1e-3)
    p = Params(nx, ny, dx, dx, cfl=0.4, h_dry=1e-3, kappa_cap=1.0)
    return Scenario(f"mitigation_{nx}x{ny}_s{seed}", p, _f32(b), _f32(n), _f32(h),
                    _f32(hu), _f32(hv), nsteps, dict(seed=seed, xs=xs))


def mitigation_ensemble(count: int = 64, nx: int = 1024, ny: int = 1024,
                        nsteps: int = 3000, seed0: int = 1000):
    """Batched ensemble on one shared grid size (seeds ``seed0 + s``)."""
    return [mitigation_coast(nx, ny, 2.0, seed0 + s, nsteps) for s in range(count)]


UNEVEN_SIZES = ((256, 256), (512, 1024), (1024, 1024), (2048, 1024))  # (nx, ny)


def uneven_plan(count: int = 200, seed: int = 2000, step_lo: int = 1000,
                step_hi: int = 4000):
    """Sizes and step counts of the uneven batch (no fields built)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.integers(0, len(UNEVEN_SIZES), size=count)
    steps = rng.integers(step_lo, step_hi + 1, size=count)
    return [(UNEVEN_SIZES[int(k)], int(s)) for k, s in zip(idx, steps)]


def uneven_scenario(s: int, plan=None, seed0: int = 2000) -> Scenario:
    """Scenario ``s`` of the uneven batch (fields seeded with ``seed0 + s``)."""
    plan = uneven_plan() if plan is None else plan
    (nx, ny), steps = plan[s]
    return mitigation_coast(nx, ny, 2.0, seed0 + s, steps)


def with_steps(sc: Scenario, nsteps: int) -> Scenario:
    return replace(sc, nsteps=int(nsteps))


def transpose(sc: Scenario) -> Scenario:
    """The same problem with x and y exchanged (hu <-> hv, dx <-> dy)."""
    p = sc.params
    bc = (p.bc[2], p.bc[3], p.bc[0], p.bc[1])
    q = replace(p, nx=p.ny, ny=p.nx, dx=p.dy, dy=p.dx, bc=bc)
    T = lambda a: np.ascontiguousarray(a.T)
    return Scenario(sc.name + "_T", q, T(sc.b), T(sc.n), T(sc.h), T(sc.hv), T(sc.hu),
                    sc.nsteps, dict(sc.meta))


def mirror_x(sc: Scenario) -> Scenario:
    """The same problem reflected in x (x -> L - x, hu -> -hu)."""
    p = sc.params
    q = replace(p, bc=(p.bc[1], p.bc[0], p.bc[2], p.bc[3]))
    M = lambda a: np.ascontiguousarray(a[:, ::-1])
    return Scenario(sc.name + "_M", q, M(sc.b), M(sc.n), M(sc.h), -M(sc.hu), M(sc.hv),
                    sc.nsteps, dict(sc.meta))


def nwave_surface(dist_offshore, A: float = 15.0, lam: float = 2000.0, origin: float = 1000.0):
    """Carrier's N-wave surface (Section 2.4, Eq. (20)) at a distance from
    the shoreline: eta = 2 (a1 exp(-k1 (x - x1)^2) - a2 exp(-k2 (x - x2)^2))
    with x1 = origin + 0.5151125 lam, x2 = origin + 0.2048 lam,
    k1 = 28.416/lam^2, k2 = 256/lam^2, a1 = A, a2 = A/3.  The printed
    second exponent lacks its minus sign; it is read as -k2 (a decaying
    trough)."""
    x = np.asarray(dist_offshore, dtype=np.float64)
    x1, x2 = origin + 0.5151125 * lam, origin + 0.2048 * lam
    k1, k2 = 28.416 / lam ** 2, 256.0 / lam ** 2
    a1, a2 = A, A / 3.0
    return 2.0 * (a1 * np.exp(-k1 * (x - x1) ** 2) - a2 * np.exp(-k2 * (x - x2) ** 2))


def nwave_beach(nx: int = 2048, ny: int = 256, dx: float = 2.0, A: float = 15.0,
                lam: float = 2000.0, slope: float = 0.1, hill: bool = True,
                hill_height: float = 8.0, hill_radius=(60.0, 25.0), seed: int = 3,
                manning: float = 0.025, nsteps: int = 0) -> Scenario:
    """Planar beach with a coastal hill hit by Carrier's N-wave (Section 2.4).

    The still shoreline sits at 0.8 Lx with the sea to the west; the bed rises
    with ``slope`` (1/10 as in the planar-beach benchmark) and is clamped at
    +20 m.  An elliptical Gaussian hill (radii along x and y) stands on the
    shoreline at a seeded y position.  The N-wave is placed with the
    printed origin of 1000 m offshore; momentum starts at zero.  Free-slip
    walls on all sides.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = _centres(nx, ny, dx, dx)
    Lx, Ly = nx * dx, ny * dx
    xs = 0.8 * Lx
    b = np.clip((X - xs) * slope, -1e9, 20.0)
    if hill:
        cy = rng.uniform(0.3, 0.7) * Ly
        b = b + hill_height * np.exp(-(((X - xs) / hill_radius[0]) ** 2 + ((Y - cy) / hill_radius[1]) ** 2))
    eta = nwave_surface(xs - X, A, lam)
    h, hu, hv = _wet_state(eta, b, 1e-3)
    p = Params(nx, ny, dx, dx, cfl=0.4, h_dry=1e-3, kappa_cap=1.0)
    return Scenario(f"nwave_beach_{nx}x{ny}", p, _f32(b), _f32(np.full((ny, nx), manning)),
                    _f32(h), _f32(hu), _f32(hv), nsteps, dict(xs=xs, A=A, lam=lam))
