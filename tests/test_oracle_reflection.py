"""The steady regular reflection of Sec. 5.2.1 in the oracle (CPU only): the exact
two-shock state the steady solution is compared with, where and why the printed scheme
turns non-physical from a sharp start, and the smoothed start that runs.

The paper reports the Mach-20 reflection reaching t = 0.2 but states neither the initial
field, dt, tau nor lambda.  From a sharp start (pre-shock below the incident shock line,
or the inflow everywhere) the printed scheme goes non-physical within a few steps for every
lambda: line III of Eq. (dis_eq1), the dispersion term, reaches two cells from a jump, and
there it adds c (1 - c^2) / 12 times the jump of every plane.  Its leading part moves the
cell's mass, momentum and energy by dt / (12 dy) times the jump of their fluxes; at Mach 20
the kinetic energy is 400 times the internal energy, so that small shift of the energy
takes most of the temperature.  A start smoothed over a few cells keeps T > 0.
"""
import math

import numpy as np
import pytest

import fdlb_inputs as fi
import oracle
from oracle import shocks

NTHR = 8


def test_reflected_state_conserves_fluxes_and_turns_the_flow_parallel():
    """The state behind the reflected shock (from the two-shock theory at gamma = 2) has
    the same mass, normal-momentum, tangential-velocity and energy fluxes through the shock
    line as the printed post-shock state of Sec. 5.2.1, and flows along the wall."""
    angle, st3 = shocks.reflected_state(fi.REFL_POST_PRINTED)
    st2 = fi.REFL_POST_PRINTED
    assert st3[2] == 0.0
    t = np.array([math.cos(angle), math.sin(angle)])   # along the shock line
    nrm = np.array([math.sin(angle), -math.cos(angle)])  # across it, from state 2 to state 3

    def fluxes(st):
        r, u, v, T = st
        w = np.array([u, v])
        wn, wt = w @ nrm, w @ t
        p = r * T
        return np.array([r * wn, r * wn * wn + p, wt, r * wn * (2.0 * T + 0.5 * (w @ w))])

    f2, f3 = fluxes(st2), fluxes(st3)
    np.testing.assert_allclose(f3, f2, rtol=1e-9)
    assert fluxes(st2)[0] > 0  # the flow crosses the line from state 2 into state 3
    assert st3[0] > st2[0] and st3[0] * st3[3] > st2[0] * st2[3]  # compressive


def test_sharp_start_localised_to_the_dispersion_term():
    """Inflow everywhere under the printed top state, 300 x 100, dx = 3e-3, dt = tau = 1e-5.
    After one step only line III has acted on row 98 (two rows under the top side: every
    other difference there is zero); its flux part alone predicts the cell's new
    temperature within 2%, and the second step takes T below zero there."""
    pre, post = fi.REFL_PRE, fi.REFL_POST_PRINTED
    p = fi.problem(300, 100, 3e-3, 1e-5, 1e-5, 20.0, ("dirichlet", "outflow", "wall", "dirichlet"), (pre, pre, pre, post))
    f0 = oracle.init_state(p, fi.uniform_fields(300, 100, pre))
    f1, bad1 = oracle.run_f(p, f0, 1, nthreads=NTHR)
    r, u, v, T = oracle.fields(p, f1)
    # flux jump of the top side's state over the inflow state, times dt / (12 dy)
    k = 1e-5 / (12 * 3e-3)
    n2, ux2, uy2, T2 = post
    n = 1.0 + k * n2 * uy2
    jx = 20.0 + k * n2 * ux2 * uy2
    jy = k * (n2 * uy2 * uy2 + n2 * T2)
    E = 200.5 + k * n2 * uy2 * (0.5 * (ux2 * ux2 + uy2 * uy2) + 2.0 * T2)
    T_pred = E / n - 0.5 * ((jx / n) ** 2 + (jy / n) ** 2)
    assert bad1 == -1
    assert abs(T[98, 150] - T_pred) < 0.02 * T_pred, (T[98, 150], T_pred)
    assert T[98, 150] < 0.4 * 0.5  # 63% of the temperature gone in one step
    f2, _ = oracle.run_f(p, f1, 1, nthreads=NTHR)
    assert oracle.fields(p, f2)[3][98, 150] < 0


@pytest.mark.parametrize("width", [0.0, 2.0])
def test_sharp_start_fails_and_smoothed_start_runs(width):
    """The paper's reflection at lambda = 20 from the staircase start goes non-physical
    within 20 steps; with the incident shock smoothed over two cells it stays physical
    (the GPU tests run it to the paper's t = 0.2)."""
    p, flds, _ = fi.paper_reflection(lam=20.0, width=width)
    f = oracle.init_state(p, flds)
    steps = 20 if width == 0.0 else 300
    f, bad = oracle.run_f(p, f, steps, nthreads=NTHR)
    if width == 0.0:
        assert bad != -1
    else:
        assert bad == -1
        T = oracle.fields(p, f)[3]
        assert T.min() > 0.4


@pytest.mark.parametrize("dt", [1e-5, 2e-6])
def test_mach20_double_mach_reflection_fails_at_the_wall_foot(dt):
    """The Mach-20 double Mach reflection of Sec. 5.2.2 (smoothed start, lambda = 20,
    dt = tau) turns non-physical first on the wall at the foot of the incident shock, a few
    cells after the wall begins at x = 0.08 (80 cells), at t of about 1.9e-4 for both time
    steps: a feature of the flow at the scheme's reading, not of the step size."""
    prob, flds, _ = fi.double_mach(mach=20.0, lam=20.0, width=2.0, dt=dt, tau=dt)
    f = oracle.init_state(prob, flds)
    first = None
    for step in range(1, int(round(3e-4 / dt)) + 1):
        f, _ = oracle.run_f(prob, f, 1, nthreads=NTHR, step0=step - 1)
        T = oracle.fields(prob, f)[3]
        bad = np.argwhere(~(T > 0))
        if len(bad):
            first = (step, bad)
            break
    assert first is not None
    step, bad = first
    assert 1.5e-4 < step * dt < 2.5e-4, step * dt
    assert all(y <= 1 and 82 <= x <= 95 for y, x in bad.tolist()), bad.tolist()
