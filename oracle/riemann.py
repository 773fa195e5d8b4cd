"""Exact solution of the one-dimensional Riemann problem for the Euler equations of an
ideal gas (test infrastructure only).

The paper compares its tube runs with "analytical solutions" (Sec. 5.1, Figs. 7-11).  The
gas of the Watari-Tsutahara model carries internal energy n T in two dimensions, so its
ratio of specific heats is gamma = 2; the solution here takes gamma as a parameter.

Method: the textbook two-rarefaction / two-shock pressure function for the star region,
solved by Newton iteration, followed by sampling of the self-similar solution at x/t
(Godunov's exact solver).  States are (rho, u, p); T = p / rho.
"""
from __future__ import annotations

import math

import numpy as np


class Vacuum(ValueError):
    pass


def _fk(p, rho, pk, ak, gamma):
    """Velocity jump across the left or right wave as a function of the star pressure, and
    its derivative."""
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        sq = math.sqrt(A / (p + B))
        return (p - pk) * sq, sq * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    e = (gamma - 1.0) / (2.0 * gamma)
    f = 2.0 * ak / (gamma - 1.0) * ((p / pk) ** e - 1.0)
    df = 1.0 / (rho * ak) * (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma=2.0, tol=1e-14, maxit=200):
    """(p*, u*) of the Riemann problem with primitive states (rho, u, p)."""
    rl, ul, pl = map(float, left)
    rr, ur, pr = map(float, right)
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    if 2.0 * (al + ar) / (gamma - 1.0) <= ur - ul:
        raise Vacuum("the initial data generate vacuum")
    # start from the two-rarefaction approximation
    e = (gamma - 1.0) / (2.0 * gamma)
    p = ((al + ar - 0.5 * (gamma - 1.0) * (ur - ul)) / (al / pl ** e + ar / pr ** e)) ** (1.0 / e)
    p = max(p, 1e-300)
    for _ in range(maxit):
        fl, dfl = _fk(p, rl, pl, al, gamma)
        fr, dfr = _fk(p, rr, pr, ar, gamma)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        if pn <= 0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, al, gamma)
    fr, _ = _fk(p, rr, pr, ar, gamma)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def _sample_vacuum(rl, ul, pl, al, rr, ur, pr, ar, xi, gamma):
    """Data that generate vacuum: a left and a right rarefaction whose tails bound a vacuum
    (rho = p = 0) between uL + 2 aL / (gamma - 1) and uR - 2 aR / (gamma - 1)."""
    g1 = (gamma - 1.0) / (gamma + 1.0)
    tl = ul + 2.0 * al / (gamma - 1.0)
    tr = ur - 2.0 * ar / (gamma - 1.0)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for idx, s in np.ndenumerate(xi):
        if s <= ul - al:
            st = (rl, ul, pl)
        elif s < tl:
            c = 2.0 / (gamma + 1.0) + g1 / al * (ul - s)
            st = (rl * c ** (2.0 / (gamma - 1.0)), 2.0 / (gamma + 1.0) * (al + 0.5 * (gamma - 1.0) * ul + s),
                  pl * c ** (2.0 * gamma / (gamma - 1.0)))
        elif s <= tr:
            st = (0.0, s, 0.0)
        elif s < ur + ar:
            c = 2.0 / (gamma + 1.0) - g1 / ar * (ur - s)
            st = (rr * c ** (2.0 / (gamma - 1.0)), 2.0 / (gamma + 1.0) * (-ar + 0.5 * (gamma - 1.0) * ur + s),
                  pr * c ** (2.0 * gamma / (gamma - 1.0)))
        else:
            st = (rr, ur, pr)
        rho[idx], u[idx], p[idx] = st
    return rho, u, p


def sample(left, right, xi, gamma=2.0):
    """Primitive state (rho, u, p) at similarity coordinates xi = (x - x0) / t."""
    rl, ul, pl = map(float, left)
    rr, ur, pr = map(float, right)
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    if 2.0 * (al + ar) / (gamma - 1.0) <= ur - ul:
        return _sample_vacuum(rl, ul, pl, al, rr, ur, pr, ar, np.asarray(xi, dtype=np.float64), gamma)
    ps, us = star_state(left, right, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for idx, s in np.ndenumerate(xi):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                sl = ul - al * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pl + (gamma - 1.0) / (2.0 * gamma))
                if s <= sl:
                    st = (rl, ul, pl)
                else:
                    st = (rl * (ps / pl + g1) / (g1 * ps / pl + 1.0), us, ps)
            else:  # left rarefaction
                shl = ul - al
                asl = al * (ps / pl) ** ((gamma - 1.0) / (2.0 * gamma))
                stl = us - asl
                if s <= shl:
                    st = (rl, ul, pl)
                elif s >= stl:
                    st = (rl * (ps / pl) ** (1.0 / gamma), us, ps)
                else:
                    c = 2.0 / (gamma + 1.0) + g1 / al * (ul - s)
                    st = (rl * c ** (2.0 / (gamma - 1.0)),
                          2.0 / (gamma + 1.0) * (al + 0.5 * (gamma - 1.0) * ul + s),
                          pl * c ** (2.0 * gamma / (gamma - 1.0)))
        else:  # right of the contact
            if ps > pr:  # right shock
                sr = ur + ar * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pr + (gamma - 1.0) / (2.0 * gamma))
                if s >= sr:
                    st = (rr, ur, pr)
                else:
                    st = (rr * (ps / pr + g1) / (g1 * ps / pr + 1.0), us, ps)
            else:  # right rarefaction
                shr = ur + ar
                asr = ar * (ps / pr) ** ((gamma - 1.0) / (2.0 * gamma))
                str_ = us + asr
                if s >= shr:
                    st = (rr, ur, pr)
                elif s <= str_:
                    st = (rr * (ps / pr) ** (1.0 / gamma), us, ps)
                else:
                    c = 2.0 / (gamma + 1.0) - g1 / ar * (ur - s)
                    st = (rr * c ** (2.0 / (gamma - 1.0)),
                          2.0 / (gamma + 1.0) * (-ar + 0.5 * (gamma - 1.0) * ur + s),
                          pr * c ** (2.0 * gamma / (gamma - 1.0)))
        rho[idx], u[idx], p[idx] = st
    return rho, u, p


def tube_solution(left_rhouT, right_rhouT, x, x0, t, gamma=2.0):
    """Exact (rho, u, T) at positions x and time t for tube data given as (rho, u, 0, T)."""
    def prim(s):
        rho, u, _, T = map(float, s)
        return (rho, u, rho * T)
    rho, u, p = sample(prim(left_rhouT), prim(right_rhouT), (np.asarray(x) - x0) / t, gamma)
    T = np.divide(p, rho, out=np.zeros_like(p), where=rho > 0)  # T = 0 in a vacuum
    return rho, u, T
