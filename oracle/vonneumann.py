"""Von Neumann analysis of the scheme (Sec. 4 of the paper) -- test infrastructure only.

Builds the 33 x 33 amplification matrix of Eq. (gi_j_eq) for a Fourier mode exp(i k x)
along x around a uniform equilibrium, with the Jacobian of Eq. (pian_fki_eq), and returns
its spectral radius.  The paper evaluated these matrices in Mathematica; here they are
evaluated with mpmath.

Readings (listed in the design notes):
  R8  the switching function theta_{alpha I} of line IV is frozen at a given value (the
      paper's figures vary lambda, which only matters if the switch is on); theta = 0 is
      the plain scheme on a smooth state;
  R9  the wave runs along x, phi = k dx in (0, pi]; the y lines vanish for it.

G is strongly non-normal at high Mach number (dfeq/df has entries ~1e5 at u = 30), so its
eigenvalues are computed at 40+ significant digits; float64 eigenvalues of the same matrix
can be wrong in the second digit.
"""
from __future__ import annotations

import mpmath as mp


def velocities(v, dps=None):
    """Velocity components of Eq. (dvm_eq_1) in mpmath (exact 0 and +-1, sqrt(2)/2 at the
    working precision)."""
    s = mp.sqrt(2) / 2
    dirs = [(s, s), (0, 1), (-s, s), (-1, 0), (-s, -s), (0, -1), (s, -s), (1, 0)]
    vx, vy = [mp.mpf(0)], [mp.mpf(0)]
    for k in range(4):
        for c, sn in dirs:
            vx.append(mp.mpf(v[k]) * c)
            vy.append(mp.mpf(v[k]) * sn)
    return vx, vy


def weights(v, T):
    """F_0..F_4 of Eqs. (fk_eq1), (f0_eq), (kl_eq)."""
    T = mp.mpf(T)
    F = [None] * 5
    for k in range(4):
        vk2 = mp.mpf(v[k]) ** 2
        a, b, d = (mp.mpf(v[(k + l) % 4]) ** 2 for l in (1, 2, 3))
        num = 48 * T ** 4 - 6 * (a + b + d) * T ** 3 + (a * b + b * d + d * a) * T ** 2 - a * b * d / 4 * T
        F[k + 1] = num / (vk2 * (vk2 - a) * (vk2 - b) * (vk2 - d))
    F[0] = 1 - 8 * (F[1] + F[2] + F[3] + F[4])
    return F


def feq(v, n, ux, uy, T, vel=None):
    """Eq. (feq_eq) with the bracket read as enclosing all five groups."""
    vx, vy = vel if vel is not None else velocities(v)
    F = weights(v, T)
    u2 = ux * ux + uy * uy
    h = 1 - u2 / (2 * T)
    out = []
    for q in range(33):
        k = 0 if q == 0 else 1 + (q - 1) // 8
        s = vx[q] * ux + vy[q] * uy
        br = (h + u2 ** 2 / (8 * T ** 2)) + s / T * h + s ** 2 / (2 * T ** 2) * h + s ** 3 / (6 * T ** 3) \
            + s ** 4 / (24 * T ** 4)
        out.append(n * F[k] * br)
    return out


def dfeq_df(v, state, vel=None):
    """d f^eq_i / d f_j at the equilibrium of ``state`` = (n, ux, uy, T), Eq. (pian_fki_eq):
    the chain rule through n = sum f, u = sum v f / n and T = sum |v - u|^2 f / (2 n)."""
    vx, vy = vel if vel is not None else velocities(v)
    n, ux, uy, T = (mp.mpf(a) for a in state)

    def comp(i, var):
        def fn(t):
            args = [n, ux, uy, T]
            args[var] = t
            return feq(v, *args, vel=(vx, vy))[i]
        return fn

    d = [[mp.diff(comp(i, var), [n, ux, uy, T][var]) for var in range(4)] for i in range(33)]
    J = mp.matrix(33, 33)
    for j in range(33):
        dn = 1
        dux = (vx[j] - ux) / n
        duy = (vy[j] - uy) / n
        dT = (((vx[j] - ux) ** 2 + (vy[j] - uy) ** 2) / 2 - T) / n
        for i in range(33):
            J[i, j] = d[i][0] * dn + d[i][1] * dux + d[i][2] * duy + d[i][3] * dT
    return J


def amplification(v, state, dx, dt, tau, phi, theta=0, lines=15, jac=None, vel=None):
    """G(phi) of Eq. (gi_j_eq) for an x wave; ``lines`` selects lines I-IV of Eq. (dis_eq1)
    as bits 0..3."""
    vx, vy = vel if vel is not None else velocities(v)
    n, ux, uy, T = (mp.mpf(a) for a in state)
    J = jac if jac is not None else dfeq_df(v, state, vel=(vx, vy))
    dtau = mp.mpf(dt) / mp.mpf(tau)
    e1, e2 = mp.expjpi(phi / mp.pi), mp.expjpi(2 * phi / mp.pi)
    em1, em2 = 1 / e1, 1 / e2
    kap = abs(ux * mp.mpf(dt) / mp.mpf(dx))
    av = mp.mpf(theta) * kap * (1 - kap) / 2
    G = mp.matrix(33, 33)
    for i in range(33):
        for j in range(33):
            G[i, j] = dtau * J[i, j]
        c = vx[i] * mp.mpf(dt) / mp.mpf(dx)
        diag = 1 - dtau
        if lines & 1:
            diag += -c / 2 * (e1 - em1)
        if lines & 2:
            diag += c ** 2 / 2 * (e1 - 2 + em1)
        if lines & 4:
            diag += c * (1 - c ** 2) / 12 * (e2 - 2 * e1 + 2 * em1 - em2)
        if lines & 8:
            diag += av * (e1 - 2 + em1)
        G[i, i] += diag
    return G


def spectral_radius(G):
    ev = mp.eig(G, left=False, right=False)
    return max(abs(e) for e in ev)


def max_growth(v, state, dx, dt, tau, phis, theta=0, lines=15, dps=50):
    """max over the given phases of the spectral radius of G(phi)."""
    with mp.workdps(dps):
        vel = velocities(v)
        J = dfeq_df(v, state, vel=vel)
        best = mp.mpf(0)
        for phi in phis:
            r = spectral_radius(amplification(v, state, dx, dt, tau, mp.mpf(phi), theta, lines, jac=J, vel=vel))
            best = max(best, r)
        return best
