"""The benchmark workload itself (Mach-10 regular reflection on 8192 x 2048, lambda = 20)
in the launch configuration bench.py times (default tiling, graph-replayed steps), against
the oracle at full size: float64 every value after 8 steps, both float32 storages on the
moments after 30 steps.  (The 10 000-step run itself is beyond the oracle; bench.py
compares the storages with each other there, beside float64's own sensitivity floor.)

The float32 bounds are derived, not measured: `f32_bounds` bounds the error that rounding
the stored values to float32 at every step can cause, from the oracle's own states (its
model is pinned on the CPU against both storages emulated on the oracle).
"""
import os
import sys

import numpy as np
import pytest

import fdlb_inputs as fi
import oracle
from f32_bounds import bounds, rel_errors

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


@pytest.fixture(scope="module")
def workload():
    prob, flds, _ = fi.reflection_8192x2048(mach=10.0, lam=20.0)
    return prob, flds


def test_benchmark_grid_f64_every_value(P, workload):
    prob, flds = workload
    say("benchmark workload f64, 8 steps, all 33 planes")
    s = P.Solver(prob, precision="f64")
    s.set_state(*flds)
    s.step(8)
    f_gpu = s.get_f()
    s.close()
    f_ref, bad = oracle.run_f(prob, oracle.init_state(prob, flds), 8, nthreads=NTHR)
    assert bad == -1
    if not np.array_equal(f_gpu, f_ref):
        n = int(np.count_nonzero(f_gpu != f_ref))
        raise AssertionError(f"{n} of {f_ref.size} values differ")


def test_benchmark_grid_float32_storages(P, workload):
    prob, flds = workload
    steps = 30
    say(f"benchmark workload f32dev and f32, {steps} steps, moments against the rounding bounds")
    f0 = oracle.init_state(prob, flds)
    fN, rbad = oracle.run_f(prob, f0, steps, nthreads=NTHR)
    assert rbad == -1
    ref = oracle.fields(prob, fN)
    B = bounds(prob, f0, fN, steps + 1)  # rounded when set and after each step
    del f0, fN
    errs = {}
    for prec in ("f32dev", "f32"):
        s = P.Solver(prob, precision=prec)
        s.set_state(*flds)
        s.step(steps)
        m = s.moments(allow_nonphys=True)
        _, bad = s.diag()
        s.close()
        assert not bad, prec
        errs[prec] = rel_errors(m, ref)
        say(prec, {k: (f"{v[0]:.2e}", f"{v[1]:.2e}") for k, v in errs[prec].items()})
    for prec, e in errs.items():
        for name in ("rho", "ux", "uy", "T"):
            (l1, linf), (b1, binf) = e[name], B[prec][name]
            assert l1 <= b1 and linf <= binf, f"{prec} {name}: rel L1 {l1:.3e} (bound {b1:.2e}), " \
                                              f"rel Linf {linf:.3e} (bound {binf:.2e})"
    # the deviation storage is at least a thousand times closer in L1 on rho and T
    for name in ("rho", "T"):
        assert errs["f32dev"][name][0] * 1e3 <= errs["f32"][name][0], errs
