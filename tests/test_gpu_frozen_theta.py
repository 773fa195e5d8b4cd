"""Theta of line IV frozen (fdlb_params.theta_fixed), as Sec. 4 freezes it to linearise the
scheme, through the HIP path: float64 equals the oracle's frozen-theta run bit for bit (single
steps and two steps per pass, with line IV kept and left out), and one GPU step linearised
around a uniform equilibrium has the amplification matrix of Eq. (gi_j_eq) as its Fourier
symbol, checked against the 30-digit mpmath build of it."""
import math
import os
import sys

import mpmath as mp
import numpy as np
import pytest

import fdlb_inputs as fi
import oracle
from oracle import vonneumann as vn

pytestmark = pytest.mark.gpu

NTHR = max(1, min(16, os.cpu_count() or 1))
V = (1.0, 1.92, 2.99, 4.49)


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0801_4169_amd as P
    return P


SIDES = [("dirichlet", "outflow", "wall", "dirichlet"), ("periodic",) * 4]


@pytest.mark.parametrize("sides", SIDES)
@pytest.mark.parametrize("tblock,lines", [(1, 15), (2, 15), (1, 7)])
def test_frozen_theta_bitwise_with_oracle(P, sides, tblock, lines):
    say("frozen theta 0.6", sides, "tblock", tblock, "lines", lines)
    nx, ny, steps = 140, 44, 5
    st = [(1.1, 0.4, -0.1, 0.9), (1.0, 0.2, 0.05, 1.1), (1.0, 0.3, 0.0, 1.0), (0.9, 0.35, -0.2, 1.2)]
    prob = fi.problem(nx, ny, 2e-3, 2e-5, 3e-5, 1.5, sides, st, lines=lines)
    flds = fi.random_fields(nx, ny, seed=5)
    s = P.Solver(prob, precision="f64", tblock=tblock, theta=0.6)
    s.set_state(*flds)
    s.step(steps)
    f_gpu = s.get_f()
    s.close()
    f_ref, bad = oracle.run_f(prob, oracle.init_state(prob, flds), steps, nthreads=NTHR,
                              theta_fixed=True, theta_value=0.6)
    assert bad == -1
    if not np.array_equal(f_gpu, f_ref):
        raise AssertionError(f"{int(np.count_nonzero(f_gpu != f_ref))} of {f_ref.size} values differ")
    # the switching function itself gives another result on these fields
    f_sw, _ = oracle.run_f(prob, oracle.init_state(prob, flds), steps, nthreads=NTHR)
    assert (lines & 8) == 0 or not np.array_equal(f_sw, f_ref)


@pytest.mark.parametrize("precision", ["f32", "f32dev"])
def test_frozen_theta_float32_storages_within_rounding_bounds(P, precision):
    """The float32 storages with theta frozen against the oracle's frozen-theta run, within
    the float32 rounding bounds derived from the oracle's states (and the storage really
    follows the frozen theta: the switching function's run lies outside them)."""
    from f32_bounds import bounds, rel_errors
    say("frozen theta 0.6", precision)
    nx, ny, steps = 140, 44, 5
    prob = fi.problem(nx, ny, 2e-3, 2e-5, 3e-5, 1.5, ("periodic",) * 4)
    flds = fi.random_fields(nx, ny, seed=5)
    s = P.Solver(prob, precision=precision, theta=0.6)
    s.set_state(*flds)
    s.step(steps)
    m = s.moments()
    s.close()
    f0 = oracle.init_state(prob, flds)
    fN, bad = oracle.run_f(prob, f0, steps, nthreads=NTHR, theta_fixed=True, theta_value=0.6)
    assert bad == -1
    B = bounds(prob, f0, fN, steps + 1, storages=(precision,))[precision]
    err = rel_errors(m, oracle.fields(prob, fN))
    for name in ("rho", "ux", "uy", "T"):
        assert err[name][0] <= B[name][0] and err[name][1] <= B[name][1], (name, err[name], B[name])
    f_sw, _ = oracle.run_f(prob, f0, steps, nthreads=NTHR)
    far = rel_errors(m, oracle.fields(prob, f_sw))
    assert any(far[k][1] > B[k][1] for k in far), (far, B)


def test_frozen_theta_per_batch_instance(P):
    """In one batch, an instance with theta frozen and one with the switching function:
    each equals its own single run, bit for bit (theta is an instance constant)."""
    say("batch: frozen and switching-function instances")
    st = [(1.1, 0.4, -0.1, 0.9), (1.0, 0.2, 0.05, 1.1), (1.0, 0.3, 0.0, 1.0), (0.9, 0.35, -0.2, 1.2)]
    cases = [(fi.problem(140, 44, 2e-3, 2e-5, 3e-5, 1.5, SIDES[0], st), fi.random_fields(140, 44, seed=31), 0.6),
             (fi.problem(96, 40, 2e-3, 2e-5, 3e-5, 1.5, SIDES[1], st), fi.random_fields(96, 40, seed=32), None)]
    b = P.BatchSolver([p for p, _, _ in cases], precision="f64", thetas=[th for _, _, th in cases])
    for i, (_, flds, _) in enumerate(cases):
        b.set_state(i, *flds)
    b.step(9)
    got = [b.moments(i) for i in range(len(cases))]
    b.close()
    for i, (prob, flds, th) in enumerate(cases):
        s = P.Solver(prob, precision="f64", theta=th)
        s.set_state(*flds)
        s.step(9)
        ref = s.moments()
        s.close()
        for a, r in zip(got[i], ref):
            assert np.array_equal(a, r), i


def test_linearised_gpu_step_is_the_amplification_matrix(P):
    """Uniform equilibrium on an 8-periodic strip (4 rows, uniform in y, so the y lines vanish
    as for a wave along x), perturbed by eps Re(w_m exp(i phi_m x)) for phi_m = 2 pi m / 8,
    m = 1, 2, 3 at once.  One GPU step at +eps and at -eps; the central difference, Fourier
    transformed along x, gives (N / 2) G(phi_m) w_m, to within O(eps^2) and rounding."""
    N, NY = 8, 4
    state = (1.0, 0.4, 0.25, 1.0)
    dx, dt, tau, theta = 3e-3, 2e-4, 4e-4, 0.7
    prob = fi.problem(N, NY, dx, dt, tau, 0.0, ("periodic",) * 4)
    f_eq = oracle.init_state(prob, fi.uniform_fields(N, NY, state))
    rng = np.random.default_rng(7)
    x = np.arange(N)
    modes = (1, 2, 3)
    w = {m: rng.standard_normal(33) + 1j * rng.standard_normal(33) for m in modes}
    pert = sum(np.real(w[m][:, None] * np.exp(1j * 2 * math.pi * m * x / N)[None, :]) for m in modes)
    eps = 1e-6
    out = {}
    for sgn in (1, -1):
        say("linearised step, eps", sgn * eps)
        s = P.Solver(prob, precision="f64", theta=theta)
        s.set_f(f_eq + sgn * eps * pert[:, None, :])
        s.step(1)
        out[sgn] = s.get_f()
        s.close()
    d = (out[1] - out[-1]) / (2 * eps)
    assert np.all(d == d[:, :1, :])  # uniform in y
    spec = np.fft.fft(d[:, 0, :], axis=1)  # sum_x d(x) exp(-i 2 pi k x / N)
    with mp.workdps(30):
        vel = vn.velocities(V)
        jac = vn.dfeq_df(V, state, vel=vel)
        for m in modes:
            G = vn.amplification(V, state, dx, dt, tau, mp.mpf(2) * mp.pi * m / N, theta=theta, jac=jac, vel=vel)
            Gm = np.array([[complex(G[i, j]) for j in range(33)] for i in range(33)])
            want = (N / 2) * (Gm @ w[m])
            err = np.max(np.abs(spec[:, m] - want)) / np.max(np.abs(want))
            assert err < 1e-7, (m, err)
