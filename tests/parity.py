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
import numpy as np

TOL_SMOOTH = 1e-5
TOL_SHOCK = 1e-4


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


def front_split_errors(gpu, ref, h_thin=5e-3, halo=2):
    """Errors with thin-film cells at wet/dry fronts treated apart.

    Where the depth is within a few h_dry of zero the solution is set-valued
    under rounding: whether a cell counts as wet, and the velocity hu/h of a
    millimetre film, flip between FP32 and FP64.  Cells with depth below
    ``h_thin`` in either result, and ``halo`` cells around them along x and y,
    form the front band.  Returns (h error over the whole grid, hu and hv
    errors outside the band, max |momentum difference| inside the band,
    fraction of cells in the band).
    """
    h, hu, hv = (np.asarray(x, np.float64) for x in gpu[:3])
    rh, rhu, rhv = (np.asarray(x, np.float64) for x in ref[:3])
    thin = (h < h_thin) | (rh < h_thin)
    band = thin.copy()
    for s in range(1, halo + 1):
        band[:, s:] |= thin[:, :-s]
        band[:, :-s] |= thin[:, s:]
        band[s:, :] |= thin[:-s, :]
        band[:-s, :] |= thin[s:, :]
    keep = ~band
    q = momentum_scale(rh[keep], rhu[keep], rhv[keep])
    e_h = rel_l2(h, rh)
    e_hu = float(np.linalg.norm((hu - rhu)[keep]) / q)
    e_hv = float(np.linalg.norm((hv - rhv)[keep]) / q)
    dm = float(max(np.abs(hu - rhu)[band].max(initial=0.0), np.abs(hv - rhv)[band].max(initial=0.0)))
    return e_h, e_hu, e_hv, dm, float(band.mean())

