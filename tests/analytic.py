"""Closed-form solutions and error norms from the paper's verification section.

These are independent of the FP64 checker and of the HIP library: they pin
the checker to what the paper and the mathematics fix.

* ``dam_break_h``: Stoker wet dam break, Section 2.1 (SWASHES form).
* ``bowl_h``, ``bowl_u``: Thacker planar parabolic bowl, Section 2.2.
* ``manning_q``: uniform friction-limited discharge, Section 2.3.
* ``rel_linf``, ``rel_l2``: the relative error norms of Section 2, Eq. (9).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq

G = 9.81


def rel_linf(hc, ha):
    """max|h_c - h_a| / max|h_a| over the domain (Section 2, Eq. (9))."""
    hc, ha = np.asarray(hc, float), np.asarray(ha, float)
    return float(np.max(np.abs(hc - ha)) / np.max(np.abs(ha)))


def rel_l2(hc, ha, dA: float = 1.0):
    """sqrt(sum (h_c - h_a)^2 dA / sum h_a^2 dA) (Section 2, Eq. (9))."""
    hc, ha = np.asarray(hc, float), np.asarray(ha, float)
    return float(np.sqrt(np.sum((hc - ha) ** 2 * dA) / np.sum(ha ** 2 * dA)))


def stoker_cm(h_l: float, h_r: float, g: float = G) -> float:
    """Middle-state celerity c_m: the root in (sqrt(g h_r), sqrt(g h_l)) of
    -8 g h_r c^2 (sqrt(g h_l) - c)^2 + (c^2 - g h_r)^2 (c^2 + g h_r) = 0."""
    cl = np.sqrt(g * h_l)

    def f(c):
        return -8.0 * g * h_r * c * c * (cl - c) ** 2 + (c * c - g * h_r) ** 2 * (c * c + g * h_r)

    lo, hi = np.sqrt(g * h_r), cl
    return float(brentq(f, lo * (1 + 1e-12), hi * (1 - 1e-12), xtol=1e-15, rtol=1e-15))


def dam_break_fronts(t: float, h_l: float, h_r: float, x0: float, g: float = G):
    cm = stoker_cm(h_l, h_r, g)
    cl = np.sqrt(g * h_l)
    x1 = x0 - t * cl
    x2 = x0 + t * (2.0 * cl - 3.0 * cm)
    x3 = x0 + t * 2.0 * cm * cm * (cl - cm) / (cm * cm - g * h_r)
    return x1, x2, x3, cm


def dam_break_h(x, t: float, h_l: float, h_r: float, x0: float, g: float = G):
    """Stoker wet dam break depth h(x, t) (Section 2.1)."""
    x = np.asarray(x, float)
    if t == 0.0:
        return np.where(x <= x0, h_l, h_r)
    x1, x2, x3, cm = dam_break_fronts(t, h_l, h_r, x0, g)
    cl = np.sqrt(g * h_l)
    h = np.full_like(x, h_r)
    h = np.where(x <= x1, h_l, h)
    fan = (x > x1) & (x <= x2)
    h = np.where(fan, 4.0 / (9.0 * g) * (cl - (x - x0) / (2.0 * t)) ** 2, h)
    h = np.where((x > x2) & (x <= x3), cm * cm / g, h)
    return h


def bowl_omega(h0: float, a: float, g: float = G) -> float:
    return float(np.sqrt(2.0 * g * h0) / a)


def bowl_h(x, t: float, h0: float, a: float, L: float, amp: float, g: float = G):
    """Thacker planar bowl depth (Section 2.2) with x-amplitude ``amp``.

    The wet interval is the positive set of the printed expression, i.e. the
    interval of half-width a centred at L/2 - amp cos(omega t).
    """
    x = np.asarray(x, float)
    w = bowl_omega(h0, a, g)
    h = -h0 * (((x - 0.5 * L + amp * np.cos(w * t)) / a) ** 2 - 1.0)
    return np.maximum(h, 0.0)


def bowl_u(t: float, h0: float, a: float, amp: float, g: float = G) -> float:
    """Uniform velocity inside the wet interval."""
    w = bowl_omega(h0, a, g)
    return float(amp * w * np.sin(w * t))


def manning_q(depth: float, slope: float, n: float) -> float:
    """Uniform unit discharge q = sqrt(slope)/n depth^(5/3) (Section 2.3)."""
    return float(np.sqrt(slope) / n * depth ** (5.0 / 3.0))


def friction_decay_q(t, q0: float, depth: float, n: float, g: float = 9.81):
    """Unit discharge of uniform flow over a flat bed slowed by Manning
    friction alone (Methods, Eq. (3) with no flux gradient or bed slope):
    dq/dt = -c q^2 with c = g n^2 / depth^(7/3) for q > 0, so
    q(t) = q0 / (1 + c q0 t)."""
    c = g * n * n / depth ** (7.0 / 3.0)
    return q0 / (1.0 + c * q0 * np.asarray(t, dtype=float))
