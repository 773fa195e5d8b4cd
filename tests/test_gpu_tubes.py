"""GPU parity on the paper's other tubes (Sec. 5.1: Lax, Sjogreen, two strong shocks) at the
paper's parameters and end times.

Float64: every row of the 4-row periodic tube equals the oracle's one-row run bit for bit
(a y-uniform tube does exactly the same operations in every row, in both codes).  The two
float32 storages: relative L1 of rho and T, and L1 of u over max |u|, against that oracle
run, below the bounds written in the test (measured values times three to ten).
"""
import os
import sys

import numpy as np
import pytest

import fdlb_inputs as fi
import oracle

pytestmark = pytest.mark.gpu

NTHR = max(1, min(16, os.cpu_count() or 1))


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


# Bounds on (rho, u, T) per storage, measured values in the comments; None: the storage
# cannot represent the tube's states and the run must be flagged non-physical.  The
# two-shock states (T up to 77 at u = 20: sum |f^eq| / n ~ 1e5) make even the deviation g
# as large as f at the initial jump, so its float32 rounding shows (2e-4 after 10 steps);
# naive float32 loses the density within 10 steps.
BOUNDS = {"lax": {"f32dev": (1e-5, 2e-5, 1e-5),      # 8.2e-7, 1.5e-6, 9.4e-7
                  "f32": (0.03, 0.03, 0.06)},         # 9.8e-3, -, 2.4e-2
          "sjogreen": {"f32dev": (1e-8, 1e-7, 3e-8),  # 1.0e-9, -, 2.7e-9
                       "f32": (2e-3, 5e-3, 6e-3)},    # 1.7e-4, -, 6.2e-4
          "two_shocks": {"f32dev": (0.03, 0.03, 0.03),  # 5.5e-3, 6.1e-3, 4.2e-3
                         "f32": None}}


@pytest.mark.parametrize("name", ["lax", "sjogreen", "two_shocks"])
def test_paper_tube(P, name):
    say("paper tube", name)
    p4, f4, n = fi.paper_tube(name, ny=4)
    p1, f1, _ = fi.paper_tube(name, ny=1)
    f_ref, bad = oracle.run_f(p1, oracle.init_state(p1, f1), n, nthreads=NTHR)
    assert bad == -1
    s = P.Solver(p4, precision="f64")
    s.set_state(*f4)
    s.step(n)
    f_gpu = s.get_f()
    s.close()
    for row in range(4):
        assert np.array_equal(f_gpu[:, row, :], f_ref[:, 0, :]), row
    ref = oracle.fields(p1, f_ref)
    for prec, bounds in BOUNDS[name].items():
        s = P.Solver(p4, precision=prec)
        s.set_state(*f4)
        s.step(n)
        m = s.moments(allow_nonphys=True)
        _, flag = s.diag()
        s.close()
        if bounds is None:
            assert flag, (name, prec)
            continue
        assert not flag, (name, prec)
        r, u, T = m[0][0], m[1][0], m[3][0]
        err = (float(np.sum(np.abs(r - ref[0][0])) / np.sum(ref[0][0])),
               float(np.mean(np.abs(u - ref[1][0])) / np.max(np.abs(ref[1][0]))),
               float(np.sum(np.abs(T - ref[3][0])) / np.sum(ref[3][0])))
        assert all(e <= b for e, b in zip(err, bounds)), (name, prec, err)


@pytest.mark.parametrize("lines,nsteps", [(15, None), (11, None), (13, None), (7, 50)])
def test_fig3_tube_with_lines_left_out_bitwise(P, lines, nsteps):
    """The Fig. 3 tube (Sec. 4) with all of Eq. (dis_eq1) and with line III (11), line II
    (13) or line IV (7) left out: float64 equals the oracle's run of the same scheme bit for
    bit over the 2000 steps (a left-out line is a zero weight on the GPU, a skipped term in
    the oracle).  Without the artificial viscosity the scheme turns non-physical at step 59,
    so that case runs 50 steps."""
    p, f, steps = fi.fig3_tube(lines=lines)
    steps = nsteps or steps
    say("fig3 tube, lines", lines, steps, "steps")
    s = P.Solver(p, precision="f64")
    s.set_state(*f)
    s.step(steps)
    f_gpu = s.get_f(allow_nonphys=True)
    s.close()
    f_ref, _ = oracle.run_f(p, oracle.init_state(p, f), steps, nthreads=NTHR)
    if not np.array_equal(f_gpu, f_ref):
        n = int(np.count_nonzero(f_gpu != f_ref))
        raise AssertionError(f"lines {lines}: {n} of {f_ref.size} values differ")
