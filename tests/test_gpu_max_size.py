"""The largest planes the library accepts, on the GPU.

float64: 16384 x 16352 cells (a 2.14 GB plane, just inside the 32-bit byte offsets of the
interior tiles); float32 and deviation storage: 16384 x 16384 (2^28 cells, the cell limit).
The state is a seeded 32 x 32 pattern repeated over a periodic grid, so after any number
of steps every cell must equal the matching cell of a 32 x 32 periodic run: the oracle's
for float64, the library's own small run for the float32 storages (the same operations per
cell), which in turn must lie within the derived float32 rounding bounds of the oracle's
small run.  Every one of the 2.7e8 cells is compared, which checks the addressing across the
whole plane.
"""
import gc
import os
import sys

import numpy as np
import pytest

import fdlb_inputs as fi
import oracle
from f32_bounds import bounds, rel_errors

pytestmark = pytest.mark.gpu

NTHR = max(1, min(16, os.cpu_count() or 1))
PERIOD = 32


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


def case(nx, ny):
    return fi.problem(nx, ny, 2e-3, 2e-5, 3e-5, 1.5, ("periodic",) * 4)


def run_big(P, precision, nx, ny, small, steps):
    import torch
    reps = (ny // PERIOD, nx // PERIOD)
    s = P.Solver(case(nx, ny), precision=precision)
    s.set_state(*[np.tile(f, reps) for f in small])
    s.step(steps)
    m = s.moments()
    s.close()
    del s
    gc.collect()
    torch.cuda.empty_cache()
    return m


def assert_tiles(big, ref, what):
    for name, a, r in zip(("rho", "ux", "uy", "T"), big, ref):
        ny, nx = a.shape
        v = a.reshape(ny // PERIOD, PERIOD, nx // PERIOD, PERIOD)
        eq = v == r[None, :, None, :]
        if not eq.all():
            bad = np.argwhere(~eq)[0]
            raise AssertionError(f"{what} {name}: {int((~eq).sum())} cells differ, first at block "
                                 f"({bad[0]}, {bad[2]}) cell ({bad[1]}, {bad[3]})")


@pytest.mark.parametrize("precision,nx,ny", [("f64", 16384, 16352), ("f32", 16384, 16384),
                                             ("f32dev", 16384, 16384)])
def test_largest_plane_repeats_the_small_run(P, precision, nx, ny):
    steps = 40  # one captured 32-step graph and 8 single steps
    small = fi.random_fields(PERIOD, PERIOD, seed=11)
    if precision == "f64":
        ref, bad = oracle.run_state(case(PERIOD, PERIOD), small, steps, nthreads=NTHR)
        assert bad == -1
    else:
        s = P.Solver(case(PERIOD, PERIOD), precision=precision)
        s.set_state(*small)
        s.step(steps)
        ref = s.moments()
        s.close()
        # the small run itself against the oracle, within the float32 rounding bounds
        p = case(PERIOD, PERIOD)
        f0 = oracle.init_state(p, small)
        fN, bad = oracle.run_f(p, f0, steps, nthreads=NTHR)
        assert bad == -1
        B = bounds(p, f0, fN, steps + 1, storages=(precision,))[precision]
        err = rel_errors(ref, oracle.fields(p, fN))
        for name in ("rho", "ux", "uy", "T"):
            assert err[name][0] <= B[name][0] and err[name][1] <= B[name][1], (precision, name, err[name], B[name])
    say(precision, f"{nx}x{ny}", steps, "steps")
    big = run_big(P, precision, nx, ny, small, steps)
    say(precision, "compare every cell")
    assert_tiles(big, ref, precision)
