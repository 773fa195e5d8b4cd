"""Pins of the oracle's model (velocity set, weights, equilibrium, moments) against facts
the paper and the mathematics fix -- closed forms and invariants, not the oracle's own
formulas.  CPU only."""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

import fdlb_inputs as fi
import oracle

V = fi.V_WT
EPS = np.finfo(np.float64).eps


def _circle_average(a, b):
    """Mean of cos^a * sin^b over a uniform angle (closed form)."""
    if a % 2 or b % 2:
        return 0.0
    return math.gamma((a + 1) / 2) * math.gamma((b + 1) / 2) / (math.pi * math.gamma((a + b) / 2 + 1))


def test_velocity_set_rest_and_speeds():
    vx, vy = oracle.velocities(V)
    assert vx[0] == 0.0 and vy[0] == 0.0
    for k in range(4):
        sp = np.hypot(vx[1 + 8 * k:9 + 8 * k], vy[1 + 8 * k:9 + 8 * k])
        np.testing.assert_allclose(sp, V[k], rtol=4 * EPS)
        # directions i pi / 4, i = 1..8 (Eq. dvm_eq_1)
        ang = np.arctan2(vy[1 + 8 * k:9 + 8 * k], vx[1 + 8 * k:9 + 8 * k])
        want = np.angle(np.exp(1j * np.pi / 4 * np.arange(1, 9)))
        np.testing.assert_allclose(ang, want, atol=1e-15)
    # axis directions are exact (a rounding of cos(pi/2) would break symmetry)
    assert vx[2] == 0.0 and vy[4] == 0.0 and vx[6] == 0.0 and vy[8] == 0.0


@pytest.mark.parametrize("rank", range(1, 9))
def test_velocity_set_isotropy(rank):
    """Sec. 2: the model is isotropic at least up to rank seven.  For each speed group the
    8-direction sum of every rank-r direction tensor equals 8 x the circle average for
    r <= 7; rank 8 is where the set stops being isotropic."""
    vx, vy = oracle.velocities(V)
    for k in range(4):
        cx = vx[1 + 8 * k:9 + 8 * k] / V[k]
        cy = vy[1 + 8 * k:9 + 8 * k] / V[k]
        devs = []
        for a in range(rank + 1):
            b = rank - a
            devs.append(abs(np.sum(cx ** a * cy ** b) - 8 * _circle_average(a, b)))
        if rank <= 7:
            assert max(devs) < 1e-14
        else:
            assert max(devs) > 1e-3


@pytest.mark.parametrize("T", [0.01, 0.5, 1.0, 22.61, 89.2775, 1000.0])
def test_weights_reproduce_gaussian_radial_moments(T):
    """The weights F_k of Eq. (fk_eq1) make the isotropic part of the equilibrium carry the
    radial moments of the two-dimensional Gaussian: 8 sum_k F_k v_k^(2m) = (2 theta)^m m!
    for m = 1..4 (and the m = 0 moment is 1 by Eq. (f0_eq))."""
    F = oracle.weights(V, T)
    vk = np.array(V)
    assert abs(F[0] + 8 * F[1:].sum() - 1.0) < 64 * EPS * (abs(F[0]) + 8 * np.abs(F[1:]).sum())
    for m in range(1, 5):
        terms = 8 * F[1:] * vk ** (2 * m)
        want = (2 * T) ** m * math.factorial(m)
        assert abs(terms.sum() - want) <= 64 * EPS * np.abs(terms).sum(), (m, terms.sum(), want)
    # m = 5 is not matched: a wrong cyclic index {k+l} would typically still fail m <= 4
    terms = 8 * F[1:] * vk ** 10
    assert abs(terms.sum() / ((2 * T) ** 5 * 120) - 1) > 1e-3


STATES = [
    (1.0, 0.0, 0.0, 1.0),                 # Sod left (Sec. 5.1.1)
    (0.125, 0.0, 0.0, 0.8),               # Sod right
    (1.3, 0.7, -0.4, 0.9),
    (2.0, 30.0, 0.0, 1.0),                # Fig. 2 state (Sec. 4)
    (1.0, 20.0, 0.0, 0.5),                # Mach-20 inflow (Sec. 5.2.1)
    (50 / 17, 16.7, -5.71578, 22.61),     # reflection post-shock state
    (1.0, 0.0, 0.0, 1000.0),              # Colella left (Sec. 5.1.4)
    (1.0, 0.0, 0.0, 0.01),                # Colella right
]


def _gauss_mom(a, m, T):
    """E[(m + sqrt(T) Z)^a] for a standard normal Z."""
    return sum(math.comb(a, j) * m ** (a - j) * T ** (j / 2) * (math.prod(range(j - 1, 0, -2)) if j else 1)
               for j in range(0, a + 1, 2))


@pytest.mark.parametrize("state", STATES)
def test_equilibrium_moments_match_maxwellian_to_third_order(state):
    """Every moment sum_q f^eq_q vx^a vy^b with a + b <= 3 equals that of the Maxwellian
    with the same (n, u, T): n, n u, n(T I + u u) and the third moments.  This is what the
    model needs to recover the Navier-Stokes system of Eqs. (ns_eq_1)-(ns3_eqq).  The
    identity is exact; the bound is float64 rounding scaled by the size of the terms."""
    n, ux, uy, T = state
    f = oracle.feq(V, n, ux, uy, T)
    vx, vy = oracle.velocities(V)
    for tot in range(4):
        for a in range(tot + 1):
            b = tot - a
            terms = f * vx ** a * vy ** b
            want = n * _gauss_mom(a, ux, T) * _gauss_mom(b, uy, T)
            assert abs(terms.sum() - want) <= 128 * EPS * np.abs(terms).sum() + 1e-300, (a, b)
    # with flow the fourth order is not matched (it does not have to be); at rest the
    # isotropic weights alone carry it
    if ux != 0.0:
        terms = f * vx ** 4
        assert abs(terms.sum() - n * _gauss_mom(4, ux, T) * _gauss_mom(0, uy, T)) > 1e-6 * n * T * T


@pytest.mark.parametrize("state", STATES)
def test_moments_recover_state(state):
    """Eqs. (n_eq)-(p_eq): the moments of f^eq give back (n, u, T), P = n T, to float64
    rounding scaled by the condition number sum |f| / n."""
    n, ux, uy, T = state
    f = oracle.feq(V, n, ux, uy, T)
    cond = np.abs(f).sum() / n
    got = oracle.moments(V, f)
    tol = 256 * EPS * cond
    assert abs(got[0] - n) <= tol * n
    assert abs(got[1] - ux) <= tol * (abs(ux) + math.sqrt(T)) * 10
    assert abs(got[2] - uy) <= tol * (abs(uy) + math.sqrt(T)) * 10
    # T is a difference E/n - u^2/2: its error also scales with 1 + u^2/T
    assert abs(got[3] - T) <= tol * 10 * (T + ux * ux + uy * uy)
    assert got[4] == got[0] * got[3]


def test_equilibrium_matches_extended_precision_evaluation():
    """The float64 equilibrium agrees with a 50-digit evaluation of the paper's bracket
    (all five groups inside, reading R1) to rounding scaled by the term sizes."""
    from oracle import vonneumann as vn
    with mp.workdps(50):
        vel = vn.velocities(V)
        for n, ux, uy, T in STATES:
            ref = vn.feq(V, mp.mpf(n), mp.mpf(ux), mp.mpf(uy), mp.mpf(T), vel=vel)
            got = oracle.feq(V, n, ux, uy, T)
            scale = float(max(abs(r) for r in ref))
            for q in range(33):
                assert abs(got[q] - float(ref[q])) <= 1e3 * EPS * scale


def test_mirror_maps_reverse_one_component():
    vx, vy = oracle.velocities(V)
    for q in range(33):
        mx, my = oracle.mirror(0, q), oracle.mirror(1, q)
        assert vx[mx] == -vx[q] and vy[mx] == vy[q]
        assert vx[my] == vx[q] and vy[my] == -vy[q]
        assert oracle.mirror(0, mx) == q and oracle.mirror(1, my) == q


def test_printed_shock_states_fix_gamma_two():
    """Sec. 5.2: the post-shock states the paper prints follow from the Rankine-Hugoniot
    conditions with gamma = 2 (internal energy n T in two dimensions)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "printed_shock_states.json")
    g = json.load(open(path))
    rr = g["regular_reflection"]
    post, pre = fi.oblique_shock_state(rr["pre"], beta_deg=rr["beta_deg"])
    for got, want, d in zip(post, rr["post_printed"], rr["digits_printed"]):
        assert abs(got - want) <= 0.5 * 10.0 ** (1 - d) * abs(want) + 1e-12, (got, want)
    dm = g["double_mach"]
    post = fi.moving_shock_state(dm["pre_rho"], dm["pre_T"], dm["mach"], dm["direction_deg"])
    for got, want, d in zip(post, dm["post_printed"], dm["digits_printed"]):
        assert abs(got - want) <= 0.5 * 10.0 ** (1 - d) * abs(want) + 1e-12, (got, want)
    # with gamma = 1.4 the printed reflection state is not reproduced
    post14, _ = fi.oblique_shock_state(rr["pre"], beta_deg=30.0, gamma=1.4)
    assert abs(post14[0] - rr["post_printed"][0]) > 0.1
