"""Seeded synthetic inputs for the FDLB hot path: workload parameters and initial fields.

This module is shared by the CPU oracle's tests and by the GPU path's tests and benchmark.
It holds none of the lattice Boltzmann arithmetic: it only builds parameter sets and the
macroscopic initial fields (rho, u_x, u_y, T) on the grid, plus the gas-dynamics jump
conditions that fix the post-shock states of the reflection problems.

Conventions
-----------
* A problem is a plain dict: ``nx, ny, dx, dy, dt, tau, lam, v, bc, bc_state`` where ``bc``
  lists the kinds of the sides (x-, x+, y-, y+) and ``bc_state`` the (rho, ux, uy, T) each
  Dirichlet side imposes.
* Fields are float64 arrays of shape (ny, nx), row-major (x fastest).
* Cell centres sit at ((i + 1/2) dx, (j + 1/2) dy).
* Density is the particle number density n (particle mass m = 1, Sec. 2 of the paper) and
  T is theta = T/m.
* The gas of the Watari-Tsutahara model has internal energy n T in two dimensions, so the
  ratio of specific heats is gamma = 2; the post-shock states printed in Sec. 5.2 of the
  paper are reproduced by the jump conditions below with that gamma.
"""
from __future__ import annotations

import math

import numpy as np

# Boundary kinds; the integer codes are the ones the C interfaces take.
PERIODIC, OUTFLOW, DIRICHLET, WALL = 0, 1, 2, 3
BC_NAMES = {"periodic": PERIODIC, "outflow": OUTFLOW, "dirichlet": DIRICHLET, "wall": WALL}

# Particle speeds v1..v4 of the discrete-velocity model used throughout the paper
# (Sec. 4, parameters of Fig. 2).
V_WT = (1.0, 1.92, 2.99, 4.49)

GAMMA_WT = 2.0


def _kind(b):
    return BC_NAMES[b] if isinstance(b, str) else int(b)


def problem(nx, ny, dx, dt, tau, lam, bc, bc_state=None, dy=None, v=V_WT, name="", lower=None, lines=15):
    """Parameter dict of one problem.  ``bc`` is four kinds (names or codes), x-, x+, y-, y+.
    ``lower`` optionally gives each side a lower segment: None, or (kind, state, split,
    split_rate); ghost cells whose centre coordinate along the side is below
    split + split_rate * t take that kind and state.  ``lines``: the terms of Eq. (dis_eq1)
    kept, bits 0..3 for lines I..IV (15: the full scheme)."""
    kinds = tuple(_kind(b) for b in bc)
    states = [(1.0, 0.0, 0.0, 1.0)] * 4 if bc_state is None else [tuple(map(float, s)) for s in bc_state]
    lo = tuple(None if g is None else (_kind(g[0]), tuple(map(float, g[1])), float(g[2]), float(g[3]))
               for g in (lower or (None,) * 4))
    return dict(name=name, nx=int(nx), ny=int(ny), dx=float(dx), dy=float(dx if dy is None else dy),
                dt=float(dt), tau=float(tau), lam=float(lam), v=tuple(map(float, v)),
                bc=kinds, bc_state=tuple(states), lower=lo, lines=int(lines))


def uniform_fields(nx, ny, state):
    rho, ux, uy, T = map(float, state)
    shape = (ny, nx)
    return (np.full(shape, rho), np.full(shape, ux), np.full(shape, uy), np.full(shape, T))


def riemann_fields(nx, ny, left, right, split=None):
    """Piecewise-constant Riemann data: cells i < split get ``left``, the others ``right``.

    The default split is nx // 2, i.e. the discontinuity sits at the middle of the tube
    between cells nx/2 - 1 and nx/2."""
    split = nx // 2 if split is None else split
    out = []
    for a, b in zip(left, right):
        row = np.where(np.arange(nx) < split, float(a), float(b))
        out.append(np.ascontiguousarray(np.broadcast_to(row, (ny, nx))).astype(np.float64))
    return tuple(out)


def smooth_random_fields(nx, ny, seed, base=(1.0, 0.3, -0.2, 1.0), amp=(0.1, 0.1, 0.1, 0.1),
                         modes=3):
    """Seeded smooth periodic perturbation of a base state (sum of a few Fourier modes)."""
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    out = []
    for b, a in zip(base, amp):
        fld = np.full((ny, nx), float(b))
        for _ in range(modes):
            kx, ky = rng.integers(0, 3, size=2)
            ph = rng.uniform(0, 2 * np.pi)
            fld += a / modes * rng.uniform(-1, 1) * np.cos(2 * np.pi * (kx * X + ky * Y) + ph)
        out.append(np.ascontiguousarray(fld))
    return tuple(out)


def random_fields(nx, ny, seed, base=(1.0, 0.3, -0.2, 1.0), amp=(0.05, 0.05, 0.05, 0.05)):
    """Seeded cell-by-cell noise around a base state (exercises every stencil weight)."""
    rng = np.random.default_rng(seed)
    return tuple(np.ascontiguousarray(float(b) + float(a) * rng.uniform(-1, 1, size=(ny, nx)))
                 for b, a in zip(base, amp))


# --------------------------------------------------------------------------------------
# Jump conditions (gamma = 2) for the reflection problems of Sec. 5.2
# --------------------------------------------------------------------------------------

def oblique_shock_state(pre, mach_n=None, beta_deg=30.0, gamma=GAMMA_WT):
    """Post-shock state behind a steady oblique shock.

    ``pre`` = (rho, u, 0, T) flows along +x.  The shock line falls from the top-left corner
    at angle beta to the x-axis; its unit normal towards the post-shock side is
    (sin beta, cos beta).  If ``mach_n`` is given, ``u`` is replaced so that the upstream
    normal Mach number equals it.  Returns (rho2, ux2, uy2, T2)."""
    rho1, u1, v1, T1 = map(float, pre)
    if v1 != 0.0:
        raise ValueError("pre-shock flow must be along x")
    beta = math.radians(beta_deg)
    c1 = math.sqrt(gamma * T1)
    if mach_n is not None:
        u1 = mach_n * c1 / math.sin(beta)
    wn1 = u1 * math.sin(beta)
    m2 = (wn1 / c1) ** 2
    r = (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p1 = rho1 * T1
    p2 = p1 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    rho2 = rho1 * r
    wn2 = wn1 / r
    wt = u1 * math.cos(beta)
    ux2 = wt * math.cos(beta) + wn2 * math.sin(beta)
    uy2 = -wt * math.sin(beta) + wn2 * math.cos(beta)
    return (rho2, ux2, uy2, p2 / rho2), (rho1, u1, 0.0, T1)


def moving_shock_state(pre_rho, pre_T, mach, direction_deg, gamma=GAMMA_WT):
    """State behind a normal shock of Mach ``mach`` running into gas at rest; the gas
    behind moves along ``direction_deg``.  Returns (rho2, ux2, uy2, T2)."""
    c1 = math.sqrt(gamma * pre_T)
    m2 = mach * mach
    r = (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = pre_rho * pre_T * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    rho2 = pre_rho * r
    speed = mach * c1 * (1.0 - 1.0 / r)
    d = math.radians(direction_deg)
    return (rho2, speed * math.cos(d), speed * math.sin(d), p2 / rho2)


def blend_states(pre, post, s):
    """Fields that pass from ``pre`` (s = 0) to ``post`` (s = 1): the conserved densities
    n, n u, n (|u|^2 / 2 + T) are mixed linearly with weight s (an array), then turned back
    into (n, ux, uy, T).  Every blend of two physical states is physical."""
    s = np.asarray(s, dtype=np.float64)
    r0, u0, v0, T0 = map(float, pre)
    r1, u1, v1, T1 = map(float, post)
    n = r0 * (1 - s) + r1 * s
    jx = r0 * u0 * (1 - s) + r1 * u1 * s
    jy = r0 * v0 * (1 - s) + r1 * v1 * s
    E = r0 * (0.5 * (u0 * u0 + v0 * v0) + T0) * (1 - s) + r1 * (0.5 * (u1 * u1 + v1 * v1) + T1) * s
    ux, uy = jx / n, jy / n
    T = E / n - 0.5 * (ux * ux + uy * uy)
    return tuple(np.ascontiguousarray(a) for a in (n, ux, uy, T))


def shock_profile(dist, width):
    """Weight of the post-shock state at signed distance ``dist`` (cells, positive on the
    post-shock side) from a shock line: a step for width 0, else the smooth profile
    (1 + tanh(dist / width)) / 2."""
    if width <= 0:
        return (np.asarray(dist) >= 0).astype(np.float64)
    return 0.5 * (1.0 + np.tanh(np.asarray(dist) / float(width)))


def reflection_fields(nx, ny, dx, pre, post, beta_deg, dy=None, width=0.0):
    """Initial field of the steady regular reflection: post-shock above the incident shock
    line y = Ly - x tan(beta) drawn from the top-left corner, pre-shock below.  ``width``
    (cells) smooths the line into a tanh profile of the conserved densities across it
    (0: a sharp staircase of cells)."""
    dy = dx if dy is None else dy
    Ly = ny * dy
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y)
    if width <= 0:
        above = Y >= Ly - X * math.tan(math.radians(beta_deg))
        return tuple(np.ascontiguousarray(np.where(above, float(b), float(a))) for a, b in zip(pre, post))
    b = math.radians(beta_deg)
    dist = (Y - (Ly - X * math.tan(b))) * math.cos(b) / dy  # normal distance in cells
    return blend_states(pre, post, shock_profile(dist, width))


# --------------------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------------------

SOD_L, SOD_R = (1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.8)        # Sec. 5.1.1
LAX_L, LAX_R = (0.445, 0.698, 0.0, 7.928), (0.5, 0.0, 0.0, 1.142)  # Sec. 5.1.2
COL_L, COL_R = (1.0, 0.0, 0.0, 1000.0), (1.0, 0.0, 0.0, 0.01)      # Sec. 5.1.4
TWO_L, TWO_R = (5.99924, 19.5975, 0.0, 76.8254), (5.99242, -6.19633, 0.0, 7.69222)  # Sec. 5.1.5
REFL_PRE = (1.0, 20.0, 0.0, 0.5)                                   # Sec. 5.2.1 inflow
REFL_POST_PRINTED = (50.0 / 17.0, 16.7, -5.71578, 22.61)           # Sec. 5.2.1 top state
DMR_PRE = (2.0, 0.0, 0.0, 0.5)                                     # Sec. 5.2.2
DMR_POST_PRINTED = (400.0 / 67.0, 13.3 * math.cos(math.radians(30.0)),
                    -13.3 * math.sin(math.radians(30.0)), 89.2775)

TUBE_BC = ("outflow", "outflow", "periodic", "periodic")


def sod_tube(nx=400, ny=4, dx=2.5e-3, dt=1e-5, tau=2e-5, lam=2.0):
    """Sod tube (Sec. 5.1.1 states) on the 400 x 4 grid, 1000 steps to t = 0.01."""
    p = problem(nx, ny, dx, dt, tau, lam, TUBE_BC, name="sod_400x4")
    return p, riemann_fields(nx, ny, SOD_L, SOD_R), 1000


# Tubes of Sec. 5.1 with the paper's parameters (the domain, not printed, is read as [0, 1])
SJO_L, SJO_R = (1.0, -2.0, 0.0, 0.4), (1.0, 2.0, 0.0, 0.4)                      # Sec. 5.1.3


def paper_tube(name, ny=4):
    """(problem, fields, steps) of a tube of Sec. 5.1 at the paper's dx, dt, tau, lambda and
    end time: "sod" (Sec. 5.1.1, t = 0.2), "lax" (5.1.2, t = 0.2), "sjogreen" (5.1.3,
    t = 0.018), "two_shocks" (5.1.5, t = 0.12)."""
    spec = {"sod": (1e-3, 1e-5, 1e-4, 2.0, 20000, SOD_L, SOD_R),
            "lax": (1e-3, 1e-5, 1e-4, 1.0, 20000, LAX_L, LAX_R),
            "sjogreen": (3e-3, 1e-5, 1e-5, 1.8, 1800, SJO_L, SJO_R),
            "two_shocks": (2e-3, 1e-5, 1e-5, 1.0, 12000, TWO_L, TWO_R)}[name]
    dx, dt, tau, lam, steps, L, R = spec
    nx = int(round(1.0 / dx))
    nx += nx % 2
    p = problem(nx, ny, dx, dt, tau, lam, TUBE_BC, name=f"{name}_{nx}x{ny}")
    return p, riemann_fields(nx, ny, L, R), steps


# Sec. 4, Fig. 3: two equal gases meeting at 10 (caption); speeds, dx, dt and tau of Fig. 2
FIG3_L = (10.0, 10.0, 0.0, 5.0)
FIG3_R = (10.0, 0.0, 0.0, 5.0)


def fig3_tube(t=0.02, lines=15, ny=4):
    """(problem, fields, steps) of the tube of Fig. 3 (Sec. 4): the caption's states and
    lambda = 2, with the speeds, dx = 3e-3 and dt = tau = 1e-5 of Fig. 2.  ``lines`` are
    the terms of Eq. (dis_eq1) kept (15: all; 11: without the dispersion term, line III).
    The domain [0, 1] (334 cells, jump at the middle) and the end time are not stated
    (reading: t = 0.02, before the shocks reach the ends)."""
    nx = 334
    p = problem(nx, ny, 3e-3, 1e-5, 1e-5, 2.0, TUBE_BC, name=f"fig3_lines{lines}_{nx}x{ny}", lines=lines)
    return p, riemann_fields(nx, ny, FIG3_L, FIG3_R), int(round(t / 1e-5))


def colella_tube(nx=4000, ny=4, dx=2.5e-4, dt=1e-6, tau=2e-6, lam=20.0):
    """Colella's explosion problem (Sec. 5.1.4 states, pressure ratio 1e5) on 4000 x 4,
    20000 steps to t = 0.02."""
    p = problem(nx, ny, dx, dt, tau, lam, TUBE_BC, name="colella_4000x4")
    return p, riemann_fields(nx, ny, COL_L, COL_R), 20000


def regular_reflection(nx, ny, dx, dt, tau, lam, pre, post, beta_deg, name):
    """Steady regular reflection (Sec. 5.2.1): Dirichlet inflow on the left and post-shock
    state on the top, reflecting wall at the bottom, outflow on the right."""
    bc = ("dirichlet", "outflow", "wall", "dirichlet")
    states = (pre, pre, pre, post)
    p = problem(nx, ny, dx, dt, tau, lam, bc, states, name=name)
    return p, reflection_fields(nx, ny, dx, pre, post, beta_deg)


def reflection_1024x256(lam=20.0, mach=10.0, mach_n=None, width=0.0, tau=1e-5):
    """Shock incident at 29 degrees on a reflecting wall, 1024 x 256 cells, dx = 1e-3,
    dt = 5e-6, tau = 1e-5, 40000 steps.  ``mach``: freestream (1, mach, 0, 0.5), the paper's
    way of naming a reflection's Mach number (Sec. 5.2.1: "Mach number 20" with a printed
    post-shock state that is the freestream Mach 20 one); ``mach_n`` instead fixes the
    shock-normal Mach number (pre-shock T = 0.5, u = mach_n c / sin 29deg).  ``width``:
    smoothing of the initial shock line in cells (see reflection_fields)."""
    if mach_n is not None:
        post, pre = oblique_shock_state((1.0, 1.0, 0.0, 0.5), mach_n=float(mach_n), beta_deg=29.0)
        tag = f"mn{mach_n:g}"
    else:
        post, pre = oblique_shock_state((1.0, float(mach), 0.0, 0.5), beta_deg=29.0)
        tag = f"m{mach:g}"
    p = regular_reflection_problem(1024, 256, 1e-3, 5e-6, tau, lam, pre, post, f"reflection_{tag}_29deg_1024x256")
    return p, reflection_fields(1024, 256, 1e-3, pre, post, 29.0, width=width), 40000


def reflection_8192x2048(lam=2.0, nx=8192, ny=2048, mach=20.0, tau=2e-6, width=0.0):
    """Freestream (1, mach, 0, 0.5) with a 30-degree incident shock (Sec. 5.2.1 has
    mach = 20), 2.048 x 0.512 domain, 8192 x 2048 cells, dx = 2.5e-4, dt = 1e-6, tau as
    given (2e-6 by default), 10000 steps; ``width`` smooths the initial shock line."""
    post, pre = oblique_shock_state((1.0, float(mach), 0.0, 0.5), beta_deg=30.0)
    p = regular_reflection_problem(nx, ny, 2.5e-4, 1e-6, tau, lam, pre, post, f"reflection_m{mach:g}_30deg_{nx}x{ny}")
    return p, reflection_fields(nx, ny, 2.5e-4, pre, post, 30.0, width=width), 10000


def regular_reflection_problem(nx, ny, dx, dt, tau, lam, pre, post, name):
    p, _ = regular_reflection(nx, ny, dx, dt, tau, lam, pre, post, 30.0, name)
    return p


# The reflections as this build runs them (readings of Sec. 5.2.1; the sharp staircase start
# and the shock-normal reading of "Mach 10" turn non-physical with the printed scheme):
#   - the initial incident shock is smoothed over two cells (tanh of the conserved densities);
#   - the paper's own grid keeps its printed dt = tau = 1e-5 with lambda = 20 (the paper's
#     value for its strongest tube, Colella's);
#   - the 8192 x 2048 Mach-20 grid takes tau = dt (as every strong-shock run of the paper
#     does) and lambda = 40: with tau = 2 dt, or lambda <= 30, it turns non-physical within
#     2000-4000 steps;
#   - "Mach 10 at 29 degrees" is freestream Mach 10, the paper's convention.
SMOOTH_WIDTH = 2.0


def paper_reflection(lam=20.0, width=SMOOTH_WIDTH):
    """The steady regular reflection of Sec. 5.2.1 at the paper's parameters: 300 x 100
    cells of 3e-3, inflow (1, 20, 0, 0.5) on the left, the printed post-shock state on the
    top, reflecting wall at the bottom, outflow on the right, dt = tau = 1e-5 (the value of
    all the paper's strong-shock runs), 20000 steps to t = 0.2."""
    p, _ = regular_reflection(300, 100, 3e-3, 1e-5, 1e-5, lam, REFL_PRE, REFL_POST_PRINTED, 30.0,
                              f"paper_reflection_m20_300x100_lam{lam:g}")
    return p, reflection_fields(300, 100, 3e-3, REFL_PRE, REFL_POST_PRINTED, 30.0, width=width), 20000


def cfg3_reflection():
    """The 1024 x 256 reflection as run: freestream Mach 10 at 29 degrees, lambda = 20,
    tau = 1e-5 as specified, smoothed start, 40000 steps."""
    return reflection_1024x256(lam=20.0, mach=10.0, width=SMOOTH_WIDTH)


def cfg5_reflection(nx=8192, ny=2048):
    """The 8192 x 2048 reflection as run: the paper's Mach-20 inflow and 30-degree shock,
    tau = dt = 1e-6, lambda = 40, smoothed start, 10000 steps."""
    return reflection_8192x2048(lam=40.0, nx=nx, ny=ny, mach=20.0, tau=1e-6, width=SMOOTH_WIDTH)


def ensemble_draws(count=256, seed=0, log_rp_max=2.0):
    """Instance table of the batched tube ensemble: (nx, pressure ratio, density ratio)
    drawn in this order per instance from ``numpy.random.default_rng(seed)``: nx uniform
    in [256, 4096], log10 of the pressure ratio uniform in [1, log_rp_max], density ratio
    uniform in [0.1, 10].

    The pressure ratio stops at 100 by default: with this scheme, random tubes above a
    ratio of about 100-300 turn non-physical (T < 0 ahead of the shock) in the float64
    oracle itself, for every tau, lambda and Courant number tried; log_rp_max=5 gives the
    full [10, 1e5] range."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nx = int(rng.integers(256, 4097))
        rp = float(10.0 ** rng.uniform(1.0, log_rp_max))
        rr = float(rng.uniform(0.1, 10.0))
        out.append((nx, rp, rr))
    return out


def ensemble_tubes(count=256, seed=0, ny=4, log_rp_max=2.0, tau_factor=1.0, lam=20.0):
    """Shock tubes on [0, 1] with left state (1, 0, 0, 1) and right density 1/r_rho,
    pressure 1/r_p (so T = r_rho / r_p); dx = 1/nx, dt = 0.004 dx (the dt/dx of the
    paper's Sod run), tau = tau_factor * dt, artificial-viscosity amplitude lam (Colella's
    value; lam=None interpolates 2 -> 20 in log r_p over [10, 1e5]); periodic in y.
    5000 steps."""
    probs = []
    for i, (nx, rp, rr) in enumerate(ensemble_draws(count, seed, log_rp_max)):
        dx = 1.0 / nx
        dt = 0.004 * dx
        lm = lam if lam is not None else 2.0 + 18.0 * math.log10(rp / 10.0) / 4.0
        right = (1.0 / rr, 0.0, 0.0, rr / rp)
        p = problem(nx, ny, dx, dt, tau_factor * dt, lm, TUBE_BC, name=f"tube{i}")
        probs.append((p, riemann_fields(nx, ny, (1.0, 0.0, 0.0, 1.0), right)))
    return probs, 5000


def double_mach(nx=500, ny=200, dx=1e-3, dt=1e-5, tau=1e-5, lam=2.0, mach=20.0, width=0.0):
    """Double Mach reflection (Sec. 5.2.2): a shock at 60 degrees to the x axis moving right
    at normal speed 20 into (2, 0, 0, 0.5); post-shock above the line
    y = sqrt(3) (x - 80 dx) - 40 t at t = 0, pre-shock below.  Sides: post-shock Dirichlet
    on the left; outflow on the right; at the bottom post-shock Dirichlet for x < 80 dx and
    a reflecting wall from there on; at the top post-shock for x below
    g(t) = 80 dx + (Ly + 40 t) / sqrt(3) and pre-shock beyond.  The paper runs 500 x 200
    cells (dx = 1e-3) for 750 steps and states no dt, tau or lambda: dt = tau = 1e-5 as in
    its other strong-shock runs, lambda as chosen.  ``mach`` != 20 runs the same geometry
    with a weaker shock: normal speed ``mach`` (the line moves as sqrt(3)(x - x0) - 2 mach t)
    and the Rankine-Hugoniot post-shock state at gamma = 2.  ``width`` (cells) smooths the
    initial shock line into a tanh profile of the conserved densities (0: sharp)."""
    pre = DMR_PRE
    post = DMR_POST_PRINTED if mach == 20.0 else moving_shock_state(pre[0], pre[3], mach, -30.0)
    x0 = 80 * dx
    Ly = ny * dx
    r3 = math.sqrt(3.0)
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(x, y)
    if width > 0:
        dist = (Y - r3 * (X - x0)) * 0.5 / dx  # normal distance to the 60-degree line, cells
        fields = blend_states(pre, post, shock_profile(dist, width))
    else:
        above = Y >= r3 * (X - x0)
        fields = tuple(np.ascontiguousarray(np.where(above, float(b), float(a))) for a, b in zip(pre, post))
    bc = ("dirichlet", "outflow", "wall", "dirichlet")
    states = (post, post, post, pre)
    lower = (None, None, ("dirichlet", post, x0, 0.0), ("dirichlet", post, x0 + Ly / r3, 2.0 * mach / r3))
    p = problem(nx, ny, dx, dt, tau, lam, bc, states, lower=lower, name=f"double_mach_m{mach:g}_{nx}x{ny}")
    return p, fields, 750

