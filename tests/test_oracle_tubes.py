"""The oracle on the paper's other tubes (Sec. 5.1: Lax, Sjogreen, two strong shocks) against
the exact Riemann solution at gamma = 2, the exact solver's vacuum branch (Sjogreen's
data generate vacuum at gamma = 2) against conservation, and the dispersion term's effect
on the tube of Fig. 3 (Sec. 4).

The paper prints no error norms, so each bound is the measured L1 difference times about
two; what the paper states in words is checked as stated (Sjogreen: density and
temperature stay positive).
"""
import os

import numpy as np
import pytest

import fdlb_inputs as fi
import oracle
from oracle import riemann

GAMMA = 2.0
NTHR = max(1, min(8, os.cpu_count() or 1))


def test_vacuum_branch_conserves_mass_momentum_energy():
    """Sjogreen's data at t = 0.1 on [-1, 1] (the waves stay inside): the integrals change
    only by the boundary fluxes of the untouched states."""
    L, R = (1.0, -2.0, 0.4), (1.0, 2.0, 0.4)  # (rho, u, p)
    t = 0.1
    x = np.linspace(-1.0, 1.0, 400001)
    r, u, p = riemann.sample(L, R, x / t, GAMMA)
    E = p / (GAMMA - 1.0) + 0.5 * r * u * u
    integ = lambda f: float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(x)))
    EL = L[2] / (GAMMA - 1.0) + 0.5 * L[0] * L[1] ** 2
    ER = R[2] / (GAMMA - 1.0) + 0.5 * R[0] * R[1] ** 2
    mass = (L[0] + R[0]) - t * (R[0] * R[1] - L[0] * L[1])
    mom = (L[0] * L[1] + R[0] * R[1]) - t * ((R[0] * R[1] ** 2 + R[2]) - (L[0] * L[1] ** 2 + L[2]))
    en = (EL + ER) - t * (R[1] * (ER + R[2]) - L[1] * (EL + L[2]))
    assert abs(integ(r) - mass) < 1e-6 and abs(integ(r * u) - mom) < 1e-6 and abs(integ(E) - en) < 1e-6
    # vacuum between the rarefaction tails u_L + 2 a_L / (gamma - 1) and u_R - 2 a_R / (gamma - 1)
    a = np.sqrt(GAMMA * 0.4)
    inside = (x / t > -2.0 + 2 * a + 1e-9) & (x / t < 2.0 - 2 * a - 1e-9)
    assert inside.any() and np.all(r[inside] == 0.0) and np.all(p[inside] == 0.0)
    assert np.all(r[~inside] >= 0.0)


def _run_vs_exact(name):
    p, f, n = fi.paper_tube(name, ny=1)
    (r, u, _, T), bad = oracle.run_state(p, f, n, nthreads=8)
    nx = p["nx"]
    x = (np.arange(nx) + 0.5) * p["dx"]
    L, R = {"lax": (fi.LAX_L, fi.LAX_R), "sjogreen": (fi.SJO_L, fi.SJO_R), "two_shocks": (fi.TWO_L, fi.TWO_R)}[name]
    re, ue, Te = riemann.tube_solution(L, R, x, (nx // 2) * p["dx"], n * p["dt"], GAMMA)
    l1 = lambda a, b: float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))
    return bad, r[0], T[0], (l1(r[0], re), float(np.mean(np.abs(u[0] - ue)) / np.max(np.abs(ue))), l1(T[0], Te))


@pytest.mark.slow
@pytest.mark.parametrize("name,bounds", [("lax", (0.03, 0.005, 0.02)),         # measured 0.014, 0.0021, 0.0098
                                         ("two_shocks", (0.1, 0.12, 0.13)),    # measured 0.050, 0.059, 0.067
                                         ("sjogreen", (0.01, 0.008, 0.07))])   # measured 0.0032, 0.0038, 0.032
def test_paper_tube_follows_exact_solution(name, bounds):
    bad, r, T, err = _run_vs_exact(name)
    assert bad == -1
    assert all(e < b for e, b in zip(err, bounds)), (name, err)
    if name == "sjogreen":
        # the paper: density and temperature stay positive near the near-vacuum centre
        assert r.min() > 0.0 and T.min() > 0.0


def test_fig3_dispersion_term_lowers_the_overshoot():
    """Sec. 4, Fig. 3: the dispersion term (line III of Eq. (dis_eq1)) damps the
    oscillations at the discontinuities.  On the Fig. 3 tube at t = 0.02 the density
    overshoot above the exact star state is 1.5 with the full scheme against 2.7 without
    line III (the exact star density is 23.68).  The L1 error against the exact solution is
    not lower with line III at this reading (0.030 against 0.028), so only the overshoot is
    pinned."""
    over = {}
    for lines in (15, 11):
        p, f, steps = fi.fig3_tube(lines=lines)
        m, bad = oracle.run_state(p, f, steps, nthreads=NTHR)
        assert bad == -1
        x = (np.arange(p["nx"]) + 0.5) * p["dx"]
        ex = riemann.tube_solution(fi.FIG3_L, fi.FIG3_R, x, 0.5 * p["nx"] * p["dx"], steps * p["dt"])
        assert abs(ex[0].max() - 23.6786) < 1e-3
        over[lines] = float(m[0][0].max() - ex[0].max())
    assert 0.0 < over[15] < 0.7 * over[11], over
