"""The float32 error bounds of `f32_bounds` against the storages emulated on the oracle: each
oracle step is followed by the rounding the storage applies (naive float32: f to float32;
deviation storage: g = f - f^eq(M) to float32 and f rebuilt from it), on a Mach-10 regular
reflection and on random periodic fields.  The emulated errors against the unrounded run must
lie under the bounds, and within a factor 1000 of them, so that a model three orders of
magnitude off in either direction fails.  Measured ratios of error to bound: 0.02 to 0.15
for every field and both storages."""
import numpy as np
import pytest

import fdlb_inputs as fi
import oracle
from f32_bounds import bounds, rel_errors

N = 20


def _round(prob, f, storage):
    if storage == "f32":
        return f.astype(np.float32).astype(np.float64)
    feq = oracle.init_state(prob, oracle.fields(prob, f))
    return feq + (f - feq).astype(np.float32).astype(np.float64)


def _emulate(prob, f0, storage):
    f = _round(prob, f0, storage)
    for _ in range(N):
        f, bad = oracle.run_f(prob, f, 1, nthreads=4)
        assert bad == -1
        f = _round(prob, f, storage)
    return oracle.fields(prob, f)


CASES = {
    "mach10_reflection_256x64": lambda: fi.reflection_8192x2048(mach=10.0, lam=20.0, nx=256, ny=64)[:2],
    "random_periodic_32x32": lambda: (fi.problem(32, 32, 2e-3, 2e-5, 3e-5, 1.5, ("periodic",) * 4),
                                      fi.random_fields(32, 32, seed=11)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_emulated_storages_lie_under_the_rounding_bounds(case):
    prob, flds = CASES[case]()
    f0 = oracle.init_state(prob, flds)
    fN, bad = oracle.run_f(prob, f0, N, nthreads=4)
    assert bad == -1
    ref = oracle.fields(prob, fN)
    B = bounds(prob, f0, fN, N + 1)  # the state is rounded at the start and after each step
    for storage in ("f32", "f32dev"):
        err = rel_errors(_emulate(prob, f0, storage), ref)
        for field in ("rho", "ux", "uy", "T"):
            for e, b, what in zip(err[field], B[storage][field], ("L1", "Linf")):
                assert 1e-3 * b <= e <= b, (case, storage, field, what, e, b)
