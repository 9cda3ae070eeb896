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

FP32 storage floor.  The state itself is stored in FP32.  In deep water the
depth's rounding (half an ulp: 3.8e-6 m at 80 m) acts as a surface-elevation
noise whose gradients, times g h, drive momentum noise of ~2e-5 m^2/s per
step that travels as waves; against the small momentum of a young wave this
is a relative error of order 1e-4 that no FP32-state solver avoids.
``fp32_storage_state`` measures it with the checker alone: the FP64 checker
advanced one step at a time with its state rounded to FP32 after each step.
Where that floor exceeds the stated bound, the bound for a momentum component
is 1.5 times the floor.
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


def fp32_storage_state(oracle_mod, sc, nsteps):
    """The checker's state after nsteps with the state rounded to FP32 after
    every step (FP64 arithmetic, FP32 storage).  Restarting the checker from
    the rounded state each step is exact for REFLECT boundaries; FIXED ghosts
    would be refrozen, so only REFLECT scenarios are accepted."""
    if any(int(k) != 0 for k in sc.params.bc):
        raise ValueError("FP32-storage floor needs reflective boundaries")
    h, hu, hv = sc.h, sc.hu, sc.hv
    for _ in range(int(nsteps)):
        o = oracle_mod.Oracle(sc.params, sc.b, sc.n, h, hu, hv)
        if o.step(1) != 0:
            raise RuntimeError("checker step failed")
        h, hu, hv = (np.asarray(a, np.float32) for a in o.state())
        o.close()
    return h, hu, hv
