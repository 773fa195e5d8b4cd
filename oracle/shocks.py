"""Exact gas-dynamics states of the shock reflections of Sec. 5.2 -- TEST INFRASTRUCTURE ONLY.

The Watari-Tsutahara gas has internal energy n T in two dimensions, so gamma = 2 (Sec. 2,
Eq. (p_eq)).  A regular reflection is two steady oblique shocks: the incident one turns the
freestream by some angle toward the wall, and the reflected one turns the flow behind it
back parallel to the wall.  `reflected_state` solves the second: given the state behind the
incident shock, it finds the weak oblique shock whose deflection cancels the flow angle
(bisection on the textbook theta-beta-Mach relation) and returns the state behind it with
the Rankine-Hugoniot jump of the normal component.  Used to check the steady solution the
scheme reaches (the paper says its reflected shock agrees with the exact solution).
"""
from __future__ import annotations

import math


def oblique_deflection(mach, beta, gamma=2.0):
    """Flow deflection of an oblique shock of angle beta (to the upstream flow) at upstream
    Mach number `mach`."""
    m2s = (mach * math.sin(beta)) ** 2
    return math.atan(2.0 / math.tan(beta) * (m2s - 1.0) / (mach * mach * (gamma + math.cos(2.0 * beta)) + 2.0))


def reflected_state(post, gamma=2.0):
    """(wall angle of the reflected shock [rad], state behind it (rho, ux, uy, T)) for the
    flow `post` = (rho, ux, uy < 0, T) behind the incident shock, moving toward a wall at
    y = 0.  The state behind has uy = 0."""
    r2, u2, v2, T2 = map(float, post)
    speed = math.hypot(u2, v2)
    mach = speed / math.sqrt(gamma * T2)
    theta = math.atan2(-v2, u2)
    lo, hi = math.asin(1.0 / mach) + 1e-12, 0.5 * math.pi
    # weak branch: the deflection grows with beta from the Mach angle up to its maximum
    bmax = lo
    for i in range(1, 2001):
        b = lo + (hi - lo) * i / 2000
        if oblique_deflection(mach, b, gamma) > oblique_deflection(mach, bmax, gamma):
            bmax = b
    if oblique_deflection(mach, bmax, gamma) < theta:
        raise ValueError("no attached reflected shock (Mach reflection)")
    hi = bmax
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if oblique_deflection(mach, mid, gamma) < theta:
            lo = mid
        else:
            hi = mid
    beta = 0.5 * (lo + hi)
    m2s = (mach * math.sin(beta)) ** 2
    ratio = (gamma + 1.0) * m2s / ((gamma - 1.0) * m2s + 2.0)
    p3 = r2 * T2 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2s - 1.0))
    r3 = r2 * ratio
    # tangential component kept, normal component divided by the density ratio; the flow
    # leaves parallel to the wall
    wn = speed * math.sin(beta) / ratio
    wt = speed * math.cos(beta)
    u3 = math.hypot(wn, wt)
    return beta - theta, (r3, u3, 0.0, p3 / r3)
