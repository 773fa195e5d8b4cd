"""Pins of the oracle's switching function, Sec. 3, Eq. (add4), and of the line-IV weight
theta |kappa| (1 - |kappa|) / 2 with kappa = u dt / dr of Eq. (add3).  CPU only.

Each case is chosen so that a plausible slip in the oracle fails it:
  - a pressure profile that is linear along x has a zero second difference, so theta = 0
    and the step does not depend on lambda at all (a first difference P+ - P- in the
    numerator, or the density or temperature in place of P = n T, would make it depend);
  - a single pressure jump gives, worked by hand, theta = lambda (P_R - P_L) / (P_R + 3 P_L)
    on the cell left of the jump, lambda (P_R - P_L) / (3 P_R + P_L) on the cell right of
    it, and zero everywhere else (a wrong denominator, a dropped absolute value, kappa in
    place of |kappa|, or lambda applied twice changes these numbers);
  - for any positive pressures |P+ - 2 P0 + P-| <= P+ + 2 P0 + P-, so theta lies in
    [0, lambda] (a denominator without the factor 2 on P0 exceeds lambda where P0
    dominates, a dropped absolute value goes negative).
The line-IV increment is isolated as the difference between one step of the full scheme
and one step without line IV (bit 3 of `lines`): lines I-III and the BGK term are the
same in both, so the difference is theta |kappa| (1 - |kappa|) / 2 times the second
difference of f, up to the rounding of the sums.
"""
import numpy as np

import fdlb_inputs as fi
import oracle

TUBE = ("outflow", "outflow", "periodic", "periodic")
WITHOUT_IV = 7  # lines I, II, III


def _line_iv_increment(p, flds):
    """(f0, increment of line IV over one step); the input state must be physical (the
    state after the step may not be: random jumps can overshoot, which is irrelevant to
    the weight of the step that was taken)."""
    f0 = oracle.init_state(p, flds)
    full, bad_a = oracle.run_f(p, f0, 1)
    no_iv, bad_b = oracle.run_f(p, f0, 1, lines=WITHOUT_IV)
    assert bad_a != 0 and bad_b != 0
    return f0, full - no_iv


def _tube_fields(n, u, T, ny=2):
    return tuple(np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (ny, len(n))))
                 for a in (n, u, np.zeros_like(n), T))


def test_linear_pressure_profile_switches_off():
    """P = n T linear in x while n and T vary on their own: theta vanishes in every cell
    whose three pressures are collinear (all but the two outflow end cells), so lambda
    changes nothing there, although the second differences of f are large."""
    nx = 40
    i = np.arange(nx, dtype=np.float64)
    n = 1.0 + 0.3 * np.sin(0.7 * i)
    P = 1.0 + 0.02 * i
    u = 0.4 + 0.1 * np.cos(i)
    flds = _tube_fields(n, u, P / n)
    outs = {}
    for lam in (0.0, 3.0):
        p = fi.problem(nx, 2, 1e-2, 5e-3, 1e-2, lam, TUBE)
        outs[lam], bad = oracle.run_f(p, oracle.init_state(p, flds), 1)
        assert bad == -1
    inner = slice(1, nx - 1)
    scale = np.max(np.abs(outs[0.0]))
    diff = np.max(np.abs(outs[3.0][:, :, inner] - outs[0.0][:, :, inner]))
    assert diff <= 1e-14 * scale, diff / scale
    # the end cells see the outflow copy (P- = P0), a kink: there lambda must act
    ends = np.max(np.abs(outs[3.0][:, :, [0, nx - 1]] - outs[0.0][:, :, [0, nx - 1]]))
    assert ends > 1e-8 * scale


def test_single_pressure_jump_worked_by_hand():
    """P = 1 left of the jump and 3 right of it (n T = 1 * 1 and 3 * 1), lambda = 1.5,
    u dt/dx = +0.2 on the left and -0.2 on the right: theta = 1.5 * 2 / 6 = 0.5 on the
    last left cell, 1.5 * 2 / 10 = 0.3 on the first right cell, 0 elsewhere; the line-IV
    weight theta |kappa| (1 - |kappa|) / 2 is 0.5 * 0.08 = 0.04 and 0.3 * 0.08 = 0.024."""
    nx, i0 = 24, 12
    dx, dt = 1e-2, 5e-3
    left = np.arange(nx) < i0
    n = np.where(left, 1.0, 3.0)
    T = np.ones(nx)
    u = np.where(left, 0.4, -0.4)  # kappa = u dt / dx = +-0.2
    p = fi.problem(nx, 2, dx, dt, 2e-2, 1.5, TUBE)
    f0, inc = _line_iv_increment(p, _tube_fields(n, u, T))
    d2 = f0[:, :, 2:] - 2.0 * f0[:, :, 1:-1] + f0[:, :, :-2]  # second difference at cells 1..nx-2
    weight = np.zeros(nx)
    weight[i0 - 1] = 0.04
    weight[i0] = 0.024
    expect = np.zeros_like(inc)
    expect[:, :, 1:-1] = weight[None, None, 1:-1] * d2
    scale = np.max(np.abs(f0))
    np.testing.assert_allclose(inc, expect, rtol=0, atol=1e-13 * scale)
    # the two weights are not lost in the rounding: the increment is large there
    assert np.max(np.abs(inc[:, :, i0 - 1])) > 1e-3 * scale
    assert np.max(np.abs(inc[:, :, i0])) > 1e-3 * scale


def test_theta_between_zero_and_lambda_on_random_pressures():
    """Random positive n and T along x (y-uniform, so only the x switch acts): the weight
    recovered from each cell's line-IV increment, divided by |kappa| (1 - |kappa|) / 2,
    lies in [0, lambda], and reaches well into that range."""
    rng = np.random.default_rng(7)
    nx, lam = 64, 2.5
    n = rng.uniform(0.05, 3.0, nx)
    T = rng.uniform(0.05, 3.0, nx)
    u = rng.uniform(-0.8, 0.8, nx)
    dx, dt = 1e-2, 5e-3
    p = fi.problem(nx, 2, dx, dt, 2e-2, lam, TUBE)
    f0, inc = _line_iv_increment(p, _tube_fields(n, u, T))
    _, ux, _, _ = oracle.fields(p, f0)
    thetas = []
    for x in range(1, nx - 1):
        d2 = f0[:, 0, x + 1] - 2.0 * f0[:, 0, x] + f0[:, 0, x - 1]
        q = int(np.argmax(np.abs(d2)))
        a = inc[q, 0, x] / d2[q]
        kap = abs(ux[0, x] * dt / dx)
        thetas.append(a / (kap * (1.0 - kap) / 2.0))
    thetas = np.array(thetas)
    assert np.all(thetas >= -1e-9), thetas.min()
    assert np.all(thetas <= lam * (1 + 1e-9)), thetas.max()
    assert thetas.max() > 0.5 * lam
