"""Pins of the oracle's update, Eq. (dis_eq1) with Eqs. (add3), (add4), and of its boundary
treatment, against invariants, exact solutions and the paper's amplification matrix
Eq. (gi_j_eq).  CPU only."""
import math

import mpmath as mp
import numpy as np
import pytest

import fdlb_inputs as fi
import oracle
from oracle import riemann
from oracle import vonneumann as vn

V = fi.V_WT
EPS = np.finfo(np.float64).eps
PER = ("periodic",) * 4


def _fields_equal_rows(a):
    return all(np.array_equal(a[j], a[0]) for j in range(a.shape[0]))


@pytest.mark.parametrize("state", [(1.0, 0.0, 0.0, 1.0), (1.3, 0.7, -0.4, 0.9), (1.0, 20.0, 0.0, 0.5),
                                   (50 / 17, 16.7, -5.71578, 22.61), (1.0, 0.0, 0.0, 1000.0)])
def test_uniform_state_is_a_fixed_point(state):
    """A uniform equilibrium is steady: every difference in lines I-IV vanishes exactly and
    the BGK term only moves f by the rounding of f^eq.  Every cell performs the same
    operations, so the state stays bitwise uniform."""
    p = fi.problem(8, 4, 1e-3, 1e-6, 2e-6, 2.0, PER)
    f0 = oracle.init_state(p, fi.uniform_fields(8, 4, state))
    f1, bad = oracle.run_f(p, f0, 20)
    assert bad == -1
    for q in range(33):
        assert np.all(f1[q] == f1[q, 0, 0])
    # each step re-derives (n, u, T) from f with relative error ~ eps * cond * (1 + u^2/T);
    # the BGK term relaxes towards f^eq of those moments, a random walk of that size
    n, ux, uy, T = state
    cond = np.abs(f0[:, 0, 0]).sum() / n
    drift = np.max(np.abs(f1 - f0)) / np.max(np.abs(f0))
    assert drift <= 20 * 64 * EPS * cond * (1 + (ux * ux + uy * uy) / T)


def test_y_uniform_data_stays_y_uniform_bitwise():
    """A tube (data varying along x only, periodic in y) stays exactly one-dimensional."""
    p, flds, _ = fi.sod_tube(nx=64, ny=4)
    out, bad = oracle.run_state(p, flds, 200)
    assert bad == -1
    for a in out:
        assert _fields_equal_rows(a)
    assert np.max(np.abs(out[2])) < 1e-15  # +-v_y terms cancel up to the rounding of the sum


def test_x_uniform_data_stays_x_uniform_bitwise():
    p = fi.problem(4, 64, 2.5e-3, 1e-5, 2e-5, 2.0, ("periodic", "periodic", "outflow", "outflow"))
    r, u, w, T = fi.riemann_fields(64, 4, fi.SOD_L, fi.SOD_R)
    flds = (r.T.copy(), w.T.copy(), u.T.copy(), T.T.copy())
    out, bad = oracle.run_state(p, flds, 200)
    assert bad == -1
    for a in out:
        assert all(np.array_equal(a[:, i], a[:, 0]) for i in range(4))


def test_transposed_problem_gives_transposed_fields():
    """Swapping x and y (and u_x with u_y, the side conditions with each other) transposes
    the solution up to rounding: the y lines of the update are the x lines turned."""
    nx, ny = 24, 20
    p = fi.problem(nx, ny, 2e-3, 2e-5, 4e-5, 1.5, ("outflow", "outflow", "periodic", "periodic"))
    flds = fi.random_fields(nx, ny, seed=5)
    pt = fi.problem(ny, nx, 2e-3, 2e-5, 4e-5, 1.5, ("periodic", "periodic", "outflow", "outflow"))
    fT = (flds[0].T.copy(), flds[2].T.copy(), flds[1].T.copy(), flds[3].T.copy())
    a, _ = oracle.run_state(p, flds, 30)
    b, _ = oracle.run_state(pt, fT, 30)
    np.testing.assert_allclose(a[0], b[0].T, rtol=1e-13)
    np.testing.assert_allclose(a[1], b[2].T, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(a[2], b[1].T, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(a[3], b[3].T, rtol=1e-13)


def test_conservation_without_artificial_viscosity():
    """With lambda = 0 on a periodic grid every line of Eq. (dis_eq1) is a difference of
    neighbouring values and the BGK term keeps the moments of f^eq, so the totals of
    n, n u and the energy are conserved to rounding.  Line IV has a cell-dependent
    coefficient and in general changes them."""
    nx, ny = 16, 12
    flds = fi.smooth_random_fields(nx, ny, seed=3)
    vx, vy = oracle.velocities(V)
    e = 0.5 * (vx * vx + vy * vy)

    def totals(f):
        return np.array([f.sum(), (vx[:, None, None] * f).sum(), (vy[:, None, None] * f).sum(),
                         (e[:, None, None] * f).sum()])

    for lam, conserved in ((0.0, True), (5.0, False)):
        p = fi.problem(nx, ny, 2e-3, 2e-5, 4e-5, lam, PER)
        f0 = oracle.init_state(p, flds)
        f1, bad = oracle.run_f(p, f0, 20)
        assert bad == -1
        d = np.abs(totals(f1) - totals(f0)) / np.abs(f0).sum()
        if conserved:
            assert np.all(d < 1e-13), d
        else:
            assert np.any(d > 1e-12), d


def _advect_error(N, axis):
    """One collision-free step (tau = infinity, lambda = 0) of smooth periodic data: every
    plane is translated by its Courant number; returns the max deviation from the exact
    translation."""
    dx = 1.0 / N
    dt = 0.1 * dx
    if axis == 0:
        p = fi.problem(N, 1, dx, dt, math.inf, 0.0, PER)
    else:
        p = fi.problem(1, N, dx, dt, math.inf, 0.0, PER)
    vx, vy = oracle.velocities(V)
    x = np.arange(N)
    f = np.empty((33, p["ny"], p["nx"]))
    exact = np.empty_like(f)
    for q in range(33):
        c = (vx[q] if axis == 0 else vy[q]) * dt / dx
        prof = 1.0 + 0.1 * np.sin(2 * np.pi * x / N + q)
        ex = 1.0 + 0.1 * np.sin(2 * np.pi * (x - c) / N + q)
        f[q] = prof.reshape(p["ny"], p["nx"])
        exact[q] = ex.reshape(p["ny"], p["nx"])
    f1, _ = oracle.run_f(p, f, 1)
    return np.max(np.abs(f1 - exact))


@pytest.mark.parametrize("axis", [0, 1])
def test_collision_free_step_is_third_order_translation(axis):
    """Lines I-III form the modified Lax-Wendroff scheme of Sec. 3: for smooth data one
    step reproduces the exact translation f(x - v dt) up to O(phi^4) (phi = k dx), i.e.
    halving phi divides the one-step error by ~16.  A missing line II leaves O(phi^2), a
    wrong sign of line III leaves O(phi^3)."""
    e = [_advect_error(N, axis) for N in (32, 64, 128)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 15.0 < r1 < 17.5 and 15.0 < r2 < 17.5, e


def _wall_vs_periodic(axis):
    nx, ny = 12, 10
    flds = fi.smooth_random_fields(nx, ny, seed=11, base=(1.0, 0.2, 0.3, 1.0))
    if axis == 1:
        bc_w = ("periodic", "periodic", "wall", "wall")
        bc_p = PER
        pw = fi.problem(nx, ny, 2e-3, 2e-5, 4e-5, 1.0, bc_w)
        pp = fi.problem(nx, 2 * ny, 2e-3, 2e-5, 4e-5, 1.0, bc_p)
        r, u, w, T = flds
        big = (np.vstack([r, r[::-1]]), np.vstack([u, u[::-1]]), np.vstack([w, -w[::-1]]), np.vstack([T, T[::-1]]))
    else:
        bc_w = ("wall", "wall", "periodic", "periodic")
        pw = fi.problem(nx, ny, 2e-3, 2e-5, 4e-5, 1.0, bc_w)
        pp = fi.problem(2 * nx, ny, 2e-3, 2e-5, 4e-5, 1.0, PER)
        r, u, w, T = flds
        big = (np.hstack([r, r[:, ::-1]]), np.hstack([u, -u[:, ::-1]]), np.hstack([w, w[:, ::-1]]),
               np.hstack([T, T[:, ::-1]]))
    a, _ = oracle.run_state(pw, flds, 25)
    b, _ = oracle.run_state(pp, big, 25)
    return a, tuple(x[:ny, :nx] for x in b)


@pytest.mark.parametrize("axis", [0, 1])
def test_wall_equals_mirrored_periodic_domain(axis):
    """Reading R11: a reflecting wall is the specular mirror about the cell face, so a box
    with walls on both sides of one axis evolves exactly like the mirror-doubled periodic
    box (up to rounding: the mirrored cells sum their velocities in another order)."""
    a, b = _wall_vs_periodic(axis)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-12)


def test_outflow_and_dirichlet_keep_matching_uniform_state():
    state = (1.0, 3.0, -1.0, 2.0)
    for bc in (("outflow",) * 4, ("dirichlet",) * 4, ("dirichlet", "outflow", "wall", "dirichlet")):
        st = state if "wall" not in bc else (1.0, 3.0, 0.0, 2.0)
        p = fi.problem(10, 8, 1e-3, 1e-5, 2e-5, 2.0, bc, [st] * 4)
        out, bad = oracle.run_state(p, fi.uniform_fields(10, 8, st), 20)
        assert bad == -1
        for a, s in zip(out, st):
            np.testing.assert_allclose(a, s, rtol=1e-12, atol=1e-12)


def test_dirichlet_ghost_feeds_inflow():
    """A Dirichlet side holding a different state drives it into the domain."""
    p = fi.problem(40, 1, 1e-2, 1e-3, 2e-3, 1.0, ("dirichlet", "outflow", "periodic", "periodic"),
                   [(2.0, 1.0, 0.0, 1.0)] + [(1.0, 0.0, 0.0, 1.0)] * 3)
    out, bad = oracle.run_state(p, fi.uniform_fields(40, 1, (1.0, 0.0, 0.0, 1.0)), 60)
    assert bad == -1
    r = out[0][0]
    assert r[0] > 1.5 and abs(r[-1] - 1.0) < 1e-3


def test_quad_build_agrees_with_float64_on_a_well_conditioned_tube():
    p, flds, _ = fi.sod_tube(nx=64, ny=1)
    a, _ = oracle.run_state(p, flds, 100)
    b, _ = oracle.run_state(p, flds, 100, quad=True)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-12)
    assert oracle._lib(True).orc_real_bytes() == 16


# ---------------------------------------------------------------------------------------
# Amplification matrix, Eq. (gi_j_eq)
# ---------------------------------------------------------------------------------------

def test_linearised_step_equals_amplification_matrix():
    """Linearising one oracle step around a uniform equilibrium on an N-periodic strip and
    taking the block Fourier transform gives the 33 x 33 matrix G(phi) that the paper
    writes down in Eq. (gi_j_eq) (theta of line IV frozen, reading R8), entry by entry.
    G here is built from the paper's Fourier symbols and the chain rule of
    Eq. (pian_fki_eq); the oracle's step is differentiated numerically."""
    N = 8
    state = (1.0, 0.4, 0.25, 1.0)
    dx, dt, tau, theta = 3e-3, 2e-4, 4e-4, 0.7
    p = fi.problem(N, 1, dx, dt, tau, 0.0, PER)
    f0 = oracle.init_state(p, fi.uniform_fields(N, 1, state))
    flat = f0.reshape(33, N)
    h = 1e-6
    J = np.zeros((33, 33, 5))  # J[q, q', d] = dS(q, cell 0) / df(q', cell d)
    for qq in range(33):
        for d in range(-2, 3):
            cell = d % N
            fp = flat.copy()
            fm = flat.copy()
            fp[qq, cell] += h
            fm[qq, cell] -= h
            sp, _ = oracle.run_f(p, fp.reshape(33, 1, N), 1, theta_fixed=True, theta_value=theta)
            sm, _ = oracle.run_f(p, fm.reshape(33, 1, N), 1, theta_fixed=True, theta_value=theta)
            J[:, qq, d + 2] = (sp.reshape(33, N)[:, 0] - sm.reshape(33, N)[:, 0]) / (2 * h)
    with mp.workdps(30):
        vel = vn.velocities(V)
        jac = vn.dfeq_df(V, state, vel=vel)
        for m in (1, 2, 3, 4):
            phi = 2 * math.pi * m / N
            Gh = sum(J[:, :, d + 2] * np.exp(1j * phi * d) for d in range(-2, 3))
            G = vn.amplification(V, state, dx, dt, tau, mp.mpf(2) * mp.pi * m / N, theta=theta, jac=jac, vel=vel)
            Gm = np.array([[complex(G[i, j]) for j in range(33)] for i in range(33)])
            err = np.max(np.abs(Gh - Gm)) / np.max(np.abs(Gm))
            assert err < 1e-7, (m, err)


# ---------------------------------------------------------------------------------------
# Exact Riemann solutions (Sec. 5.1)
# ---------------------------------------------------------------------------------------

def test_exact_riemann_solver_textbook_case():
    """Sod's problem at gamma = 1.4 has the textbook star state p* = 0.30313, u* = 0.92745,
    and the gamma = 2 star state satisfies the shock jump conditions."""
    ps, us = riemann.star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), gamma=1.4)
    assert abs(ps - 0.30313) < 5e-5 and abs(us - 0.92745) < 5e-5
    g = 2.0
    ps, us = riemann.star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), gamma=g)
    rho, u, pr = riemann.sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), np.array([us + 1e-9]), g)
    # mass and momentum fluxes across the right shock (speed from the mass balance)
    r1, u1, p1 = 0.125, 0.0, 0.1
    r2, u2, p2 = rho[0], u[0], pr[0]
    S = (r2 * u2 - r1 * u1) / (r2 - r1)
    mom = (r2 * u2 * u2 + p2 - (r1 * u1 * u1 + p1)) - S * (r2 * u2 - r1 * u1)
    e1 = p1 / (g - 1) + 0.5 * r1 * u1 * u1
    e2 = p2 / (g - 1) + 0.5 * r2 * u2 * u2
    en = (u2 * (e2 + p2) - u1 * (e1 + p1)) - S * (e2 - e1)
    assert abs(mom) < 1e-10 and abs(en) < 1e-10


def _sod_l1(N, t_end=0.1):
    dx = 1.0 / N
    dt = 0.004 * dx
    p = fi.problem(N, 1, dx, dt, 2 * dt, 2.0, fi.TUBE_BC)
    flds = fi.riemann_fields(N, 1, fi.SOD_L, fi.SOD_R)
    nsteps = int(round(t_end / dt))
    (r, u, w, T), bad = oracle.run_state(p, flds, nsteps, nthreads=4)
    assert bad == -1
    x = (np.arange(N) + 0.5) * dx
    re, ue, Te = riemann.tube_solution(fi.SOD_L, fi.SOD_R, x, 0.5, nsteps * dt)
    return np.mean(np.abs(r[0] - re)), np.mean(np.abs(u[0] - ue)), np.mean(np.abs(T[0] - Te))


def test_sod_tube_converges_to_exact_solution():
    """Sec. 5.1.1: the Sod tube approaches the exact gamma = 2 Riemann solution as dx, dt
    and tau shrink together (dt = 0.004 dx, tau = 2 dt, lambda = 2)."""
    errs = [_sod_l1(N) for N in (100, 200, 400)]
    for k in range(3):
        assert errs[1][k] < 0.8 * errs[0][k] and errs[2][k] < 0.8 * errs[1][k], errs
    assert errs[2][0] < 0.01, errs


# --------------------------------------------------------------------------------------
# Side segments (the double Mach reflection of Sec. 5.2.2): a side whose condition changes
# at a point that may move with time.
# --------------------------------------------------------------------------------------
SEG_STATES = [(1.1, 0.4, -0.1, 0.9), (0.9, -0.2, 0.3, 1.2), (1.0, 0.1, 0.2, 1.1), (1.2, 0.0, -0.3, 0.8)]


def _seg_problem(lower, bc=("dirichlet", "outflow", "wall", "dirichlet")):
    return fi.problem(24, 16, 2e-3, 2e-5, 3e-5, 1.5, bc, SEG_STATES, lower=lower)


def test_segment_equal_to_its_side_changes_nothing():
    """A lower segment with the side's own condition, at any split, leaves every bit as it
    was."""
    flds = fi.random_fields(24, 16, seed=5)
    base = _seg_problem(None)
    same = _seg_problem(tuple((k, st, 0.013, 0.7) for k, st in zip(base["bc"], SEG_STATES)))
    a, _ = oracle.run_state(base, flds, 15)
    b, _ = oracle.run_state(same, flds, 15)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("where", ["below", "beyond"])
def test_segment_beyond_the_side_replaces_it(where):
    """A split below every cell centre leaves the side's own condition; one beyond every
    cell gives the lower condition everywhere, the same as a side of that condition."""
    flds = fi.random_fields(24, 16, seed=6)
    lo_kinds = ("wall", "dirichlet", "outflow", "wall")
    lo_states = [SEG_STATES[(k + 1) % 4] for k in range(4)]
    split = -1.0 if where == "below" else 1.0
    seg = _seg_problem(tuple((lo_kinds[k], lo_states[k], split, 0.0) for k in range(4)))
    ref = _seg_problem(None) if where == "below" else _seg_problem(
        None, bc=lo_kinds) | {"bc_state": tuple(lo_states)}
    a, _ = oracle.run_state(seg, flds, 15)
    b, _ = oracle.run_state(ref, flds, 15)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_moving_segment_restarts_at_its_time():
    """A moving split: 20 steps equal 8 steps and then 12 more started at step 8 (the time
    is (step0 + step) dt), and differ from the same split held still."""
    flds = fi.random_fields(24, 16, seed=7)
    lower = (None, None, ("dirichlet", SEG_STATES[1], 0.01, 500.0), ("wall", SEG_STATES[0], 0.03, -800.0))
    p = _seg_problem(lower)
    f0 = oracle.init_state(p, flds)
    a, _ = oracle.run_f(p, f0, 20)
    b, _ = oracle.run_f(p, f0, 8)
    b, _ = oracle.run_f(p, b, 12, step0=8)
    assert np.array_equal(a, b)
    still = _seg_problem((None, None, ("dirichlet", SEG_STATES[1], 0.01, 0.0), ("wall", SEG_STATES[0], 0.03, 0.0)))
    c, _ = oracle.run_f(still, f0, 20)
    assert not np.array_equal(a, c)


@pytest.mark.slow
def test_double_mach_reflection_readings():
    """The double Mach reflection (Sec. 5.2.2, 500 x 200, 750 steps, dt = tau = 1e-5): the
    paper's Mach-20 shock turns the state non-physical after the first step (as the Mach-20
    regular reflection does); the same geometry with a Mach-5 shock and lambda = 20 stays
    physical to the end."""
    p, f, n = fi.double_mach(lam=20.0)
    _, bad = oracle.run_state(p, f, 3, nthreads=8)
    assert bad == 1
    p, f, n = fi.double_mach(mach=5.0, lam=20.0)
    (r, _, _, T), bad = oracle.run_state(p, f, n, nthreads=8)
    assert bad == -1 and r.min() > 0 and T.min() > 0
