"""Parity metrics between the FP32 HIP path and the FP64 checker.

Tolerances (relative L2 per field): 1e-5 on smooth, fully wet problems and
1e-4 with shocks or wet/dry fronts.  These follow from FP32 arithmetic: the
state carries a relative rounding of ~6e-8 per operation; a step applies a few
hundred operations per cell whose errors mostly cancel, and the WENO weights
amplify them near discontinuities by ~1/(eps + beta) sensitivity, so smooth
runs of up to a few hundred steps stay near 1e-6 and shock or front runs near
1e-5.  Momentum components are measured against the norm of the reference momentum
field ||(hu, hv)||: a component that is nearly zero (hv of a wave travelling
in x) would otherwise divide rounding by nearly nothing.  Where the whole
momentum field vanishes the denominator falls back to 1e-6 x ||h||
sqrt(g max h), the momentum scale of a shallow-water wave on that depth.

FP32 storage.  A state stored in FP32 rounds every cell once per stage.  A
stored depth of 80 m has an ulp of 7.6e-6 m: in deep water that rounding
acts as surface noise whose gradients move the momentum by ~2e-5 m^2/s per
step (2.4e-4 of a young wave's momentum after 20 steps on the coastline) and
loses sub-ulp increments with a consistent sign (mass drift).  The GPU path
stores the level h + min(b, 0) instead, the surface elevation at sea, whose
rounding is tens of times finer; the bounds above then hold on the deep-water
coastline too.
"""
from typing import NamedTuple

import numpy as np

TOL_SMOOTH = 1e-5
TOL_SHOCK = 1e-4
# Wet/dry fronts.  A cell whose depth lies within rounding of the threshold
# h_dry = 1e-3 m may be wet in one result and dry in the other; the dry one
# has zero momentum, the wet one h |u| <~ 1e-3 m x 1 m/s.  Inside the band of
# such cells the momentum difference is bounded by TOL_BAND (m^2/s); over the
# whole grid the few band cells add at most TOL_FULL to the relative L2 of
# the momentum.
TOL_BAND = 1e-3
TOL_FULL = 1e-3


def rel_l2(a, ref, floor=0.0):
    a = np.asarray(a, np.float64)
    ref = np.asarray(ref, np.float64)
    den = max(np.linalg.norm(ref), floor)
    if den == 0.0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - ref) / den)


def momentum_scale(rh, rhu, rhv, g=9.81):
    q = np.sqrt(np.linalg.norm(rhu) ** 2 + np.linalg.norm(rhv) ** 2)
    return max(q, 1e-6 * np.linalg.norm(rh) * np.sqrt(g * max(rh.max(), 1e-12)))


def field_errors(gpu, ref, g=9.81):
    """Relative L2 errors of h and of the two momentum components."""
    h, hu, hv = (np.asarray(x, np.float64) for x in gpu[:3])
    rh, rhu, rhv = (np.asarray(x, np.float64) for x in ref[:3])
    q = momentum_scale(rh, rhu, rhv, g)
    return (rel_l2(h, rh), float(np.linalg.norm(hu - rhu) / q), float(np.linalg.norm(hv - rhv) / q))


class FrontErrors(NamedTuple):
    h: float          # relative L2 of h over the whole grid
    hu: float         # relative L2 of hu outside the front band
    hv: float         # relative L2 of hv outside the front band
    band_dq: float    # max |momentum difference| inside the band (m^2/s)
    band_frac: float  # fraction of the grid in the band
    hu_full: float    # relative L2 of hu over the whole grid
    hv_full: float    # relative L2 of hv over the whole grid
    flips: int        # cells whose wet/dry class differs


def front_split_errors(gpu, ref, h_dry=1e-3, halo=2) -> FrontErrors:
    """Errors with the cells at wet/dry fronts whose class flipped treated apart.

    A cell is wet iff its depth exceeds h_dry.  Where the depth is within
    rounding of h_dry the class is set-valued: the FP32 and FP64 results may
    disagree about it, and one of them then zeroes the momentum the other
    keeps.  Cells whose class differs between the two results, and ``halo``
    cells around them along x and y (the reach of the momentum they feed
    into the next fluxes within a step), form the front band.  Momentum
    errors are reported outside the band (relative L2), inside it (max
    absolute difference) and over the whole grid (relative L2).
    """
    h, hu, hv = (np.asarray(x, np.float64) for x in gpu[:3])
    rh, rhu, rhv = (np.asarray(x, np.float64) for x in ref[:3])
    flip = (h > h_dry) != (rh > h_dry)
    band = flip.copy()
    for s in range(1, halo + 1):
        band[:, s:] |= flip[:, :-s]
        band[:, :-s] |= flip[:, s:]
        band[s:, :] |= flip[:-s, :]
        band[:-s, :] |= flip[s:, :]
    keep = ~band
    q = momentum_scale(rh, rhu, rhv)
    qk = momentum_scale(rh[keep], rhu[keep], rhv[keep]) if keep.any() else q
    dm = float(max(np.abs(hu - rhu)[band].max(initial=0.0), np.abs(hv - rhv)[band].max(initial=0.0)))
    return FrontErrors(rel_l2(h, rh),
                       float(np.linalg.norm((hu - rhu)[keep]) / qk),
                       float(np.linalg.norm((hv - rhv)[keep]) / qk),
                       dm, float(band.mean()),
                       float(np.linalg.norm(hu - rhu) / q), float(np.linalg.norm(hv - rhv) / q),
                       int(flip.sum()))


def assert_front_parity(gpu, ref, tol, label="", h_dry=1e-3) -> FrontErrors:
    """Parity with wet/dry fronts: ``tol`` on h and, outside the front band,
    on hu and hv; TOL_BAND inside the band; TOL_FULL on the whole momentum
    field."""
    e = front_split_errors(gpu, ref, h_dry)
    print(f"front parity {label}: {e}", flush=True)
    assert max(e.h, e.hu, e.hv) <= tol, e
    assert e.band_dq <= TOL_BAND, e
    assert max(e.hu_full, e.hv_full) <= TOL_FULL, e
    return e


# Epilogue reductions.  The FP64 mass of the FP32 state differs from the
# checker's by the state's rounding (relative ~6e-8 per cell, averaging out
# over the grid) plus the FP32 drift of a few 1e-10 per step: 1e-6 of the
# mass bounds both over the runs compared here.  The clamped mass is a sum of
# deficits of films near zero depth, compared against the same 1e-6 of the
# mass.  The runup is the highest bed of a wet land cell; a film at the front
# may be wet in one result and dry in the other, so the two may name
# neighbouring cells: they agree within one cell's elevation step.
TOL_MASS = 1e-6


def bed_step(b):
    """Largest bed difference between neighbouring cells of which one is land."""
    b = np.asarray(b, np.float64)
    ex = np.abs(np.diff(b, axis=1))[(b[:, 1:] > 0) | (b[:, :-1] > 0)]
    ey = np.abs(np.diff(b, axis=0))[(b[1:, :] > 0) | (b[:-1, :] > 0)]
    return float(max(ex.max(initial=0.0), ey.max(initial=0.0)))


def film_mass(gpu, ref, sc, h_dry=1e-3):
    """Mass by which the two results differ in cells that are dry (depth at
    most h_dry) in both: films below the threshold carry no momentum and
    grow or vanish by increments that FP32 does not resolve next to a wet
    cell's level, so that mass is set-valued under rounding."""
    h = np.asarray(gpu[0], np.float64)
    rh = np.asarray(ref[0], np.float64)
    dry = (h <= h_dry) & (rh <= h_dry)
    return float(np.abs(h - rh)[dry].sum()) * sc.params.dx * sc.params.dy


def assert_epilogue_parity(st, rs, sc, label="", films=0.0):
    """FP64 mass, clamped mass and runup of a GPU read against the checker.
    ``films`` (from film_mass) widens the mass bounds by the mass of the
    sub-threshold films on which the two results differ."""
    step = bed_step(sc.b)
    print(f"epilogue {label}: mass {st['mass']!r} / {rs['mass']!r}, clamp {st['clamp_mass']!r} / "
          f"{rs['clamp_mass']!r}, runup {st['runup']!r} / {rs['runup']!r} (bed step {step:.3g}, "
          f"films {films:.3g})", flush=True)
    m = rs["mass"]
    assert abs(st["mass"] - m) <= TOL_MASS * m + films
    assert abs(st["clamp_mass"] - rs["clamp_mass"]) <= TOL_MASS * m + films
    assert abs(st["runup"] - rs["runup"]) <= step
