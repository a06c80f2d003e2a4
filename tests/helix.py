"""Closed-form helix in a sector frame, written from the circle's centre.

Test-only and independent of both trackers: where the trackers step a
state with a chord formula, this module places the particle on its circle
around an explicit centre and measures arc lengths as angles around it.

State at local x: (y, z, sin phi, tan lambda, q/pT); kappa = c*Bz*q/pT,
d(phi)/ds = -kappa; the particle moves towards larger x (cos phi > 0).
"""
import math

import numpy as np

C_LIGHT = 0.00299792458


def at_x(x1, st, x2, bz):
    """State of the same particle at local x2 (None if the circle misses x2)."""
    y1, z1, sp, tl, qpt = (float(v) for v in st)
    kap = C_LIGHT * bz * qpt
    cp = math.sqrt(1.0 - sp * sp)
    if kap == 0.0:
        dx = x2 - x1
        return np.array([y1 + dx * sp / cp, z1 + tl * dx / cp, sp, tl, qpt])
    # centre: P - C = (1/kappa)(-sin phi, cos phi)
    cx = x1 + sp / kap
    cy = y1 - cp / kap
    r2 = 1.0 / (kap * kap) - (x2 - cx) ** 2
    if r2 < 0:
        return None
    y2 = cy + math.copysign(math.sqrt(r2), kap)      # branch with cos phi > 0
    sp2 = -kap * (x2 - cx)
    cp2 = kap * (y2 - cy)
    phi1 = math.atan2(sp, cp)
    phi2 = math.atan2(sp2, cp2)
    s = (phi1 - phi2) / kap
    return np.array([y2, z1 + tl * s, sp2, tl, qpt])


def hits(x0, st, xs, bz):
    """(y, z) of the particle at each x in xs."""
    out = np.array([at_x(x0, st, x, bz)[:2] for x in xs])
    return out[:, 0], out[:, 1]
