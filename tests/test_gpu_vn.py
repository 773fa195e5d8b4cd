"""The GPU stability sweep (fdlb_vn_sweep, fdlb_vn_matrix: Sec. 4, Eqs. gi_j_eq and
pian_fki_eq, in double-double arithmetic) against oracle.vonneumann, the mpmath tool: the
amplification matrix entry by entry at 40 digits, its spectral radius at 40 digits on the
states of Figs. 2, 4, 5 and 6, and the orderings Sec. 4 states, now from the GPU values."""
import sys

import mpmath as mp
import numpy as np
import pytest

from oracle import vonneumann as vn

pytestmark = pytest.mark.gpu

V = (1.0, 1.92, 2.99, 4.49)
FIG2 = (2.0, 30.0, 0.0, 1.0)
DX, DT, TAU = 3e-3, 1e-5, 1e-5


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0801_4169_amd as P
    return P.B


def mp_radius(state, phi, theta, lines, dx=DX, dt=DT, tau=TAU, dps=40):
    with mp.workdps(dps):
        vel = vn.velocities(V)
        J = vn.dfeq_df(V, state, vel=vel)
        G = vn.amplification(V, state, dx, dt, tau, mp.mpf(phi), theta, lines, jac=J, vel=vel)
        return vn.spectral_radius(G)


@pytest.mark.parametrize("state,phi,theta,lines", [(FIG2, 1.6, 0.5, 15), ((1.0, 0.4, -0.3, 1.2), 0.7, 1.5, 15),
                                                   ((2.0, 5.0, 0.0, 25.0), 2.9, 0.0, 5)])
def test_matrix_entries_match_mpmath(B, state, phi, theta, lines):
    say("vn matrix", state, phi, theta, lines)
    g = B.fdlb_vn_matrix(B.vn_case(state, DX, DT, TAU, theta, lines, V), phi)
    with mp.workdps(40):
        vel = vn.velocities(V)
        G = vn.amplification(V, state, DX, DT, TAU, mp.mpf(phi), theta, lines, vel=vel)
        scale = max(abs(G[i, j]) for i in range(33) for j in range(33))
        worst = mp.mpf(0)
        for i in range(33):
            for j in range(33):
                re = mp.mpf(g[i, j, 0]) + mp.mpf(g[i, j, 1])
                im = mp.mpf(g[i, j, 2]) + mp.mpf(g[i, j, 3])
                worst = max(worst, abs(mp.mpc(re, im) - G[i, j]))
    assert worst / scale < 1e-27, float(worst / scale)


CASES = [  # (state, phi, theta, lines): Figs. 2 (cases i-iv), 4, 5, 6
    (FIG2, 1.2, 0.5, 1), (FIG2, 1.2, 0.5, 3), (FIG2, 1.2, 0.5, 5), (FIG2, 0.2, 0.5, 15),
    (FIG2, 1.6, 0.05, 15), (FIG2, 1.6, 3.0, 15), ((2.0, 5.0, 0.0, 1.0), 0.05, 0.0, 15),
    ((2.0, 5.0, 0.0, 25.0), 0.05, 0.0, 15), ((2.0, 10.0, 0.0, 1.0), 1.6, 0.0, 15),
]


def test_spectral_radius_matches_mpmath(B):
    say("vn sweep against mpmath on", len(CASES), "cases")
    cases = [B.vn_case(s, DX, DT, TAU, th, ln, V) for s, _, th, ln in CASES]
    phis = sorted({p for _, p, _, _ in CASES})
    r = B.fdlb_vn_sweep(cases, phis)
    assert np.all(np.isfinite(r))
    for c, (s, p, th, ln) in enumerate(CASES):
        ref = mp_radius(s, p, th, ln)
        got = r[c, phis.index(p)]
        assert abs(got - float(ref)) < 1e-12 * float(ref), (s, p, th, ln, got, float(ref))


def test_float64_eigenvalues_are_wrong_where_the_gpu_sweep_is_right(B):
    """The reason for double-double: numpy's float64 eigenvalues of the Fig. 2 matrix (iv)
    miss the 40-digit spectral radius by far more than the GPU value does."""
    s, p, th, ln = FIG2, 0.13, 0.5, 15
    g = B.fdlb_vn_matrix(B.vn_case(s, DX, DT, TAU, th, ln, V), p)
    G64 = (g[..., 0] + g[..., 1]) + 1j * (g[..., 2] + g[..., 3])
    r64 = float(np.max(np.abs(np.linalg.eigvals(G64))))
    rg = B.fdlb_vn_sweep([B.vn_case(s, DX, DT, TAU, th, ln, V)], [p])[0, 0]
    ref = float(mp_radius(s, p, th, ln))
    assert abs(rg - ref) < 1e-12 and abs(r64 - ref) > 1e-6, (rg, r64, ref)


def test_orderings_of_sec4_from_the_gpu(B):
    """Figs. 2, 4, 5, 6 as Sec. 4 states them, over a phase scan on the GPU: dissipation
    (line II) stabilises, dispersion (line III) destabilises, the switch brings the full
    scheme to about 1; larger lambda lowers the growth within the plotted range; higher T
    is more stable; higher u less stable."""
    say("vn orderings from a phase scan")
    phis = np.linspace(np.pi / 64, np.pi, 64)

    def g(state, theta, lines):
        return B.fdlb_vn_sweep([B.vn_case(state, DX, DT, TAU, theta, lines, V)], phis)[0].max()

    i, ii, iii, iv = (g(FIG2, 0.5, ln) for ln in (1, 3, 5, 15))
    assert iii > i > ii > iv and abs(iv - 1.0) < 2e-4
    lam = [g(FIG2, t, 15) for t in (0.05, 0.1, 1.0, 3.0)]
    assert lam[0] > lam[1] > 1.0 > lam[2] > lam[3]
    assert g((2.0, 5.0, 0.0, 1.0), 0.0, 15) > g((2.0, 5.0, 0.0, 25.0), 0.0, 15)
    us = [g((2.0, u, 0.0, 1.0), 0.0, 15) for u in (0.0, 10.0, 30.0)]
    assert us[0] < 1.0 < us[1] < us[2]
