"""The allocation-free diagnostics entry point (fdlb_diag_noalloc) against fdlb_diag,
through the C interface: the same totals bit for bit and the same flag, on two calls in a
row with different contexts (the second smaller), on a batch, and the size limit of its
fixed scratch."""
import sys

import numpy as np
import pytest

import fdlb_inputs as fi

pytestmark = pytest.mark.gpu


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


def _both(B, ctx):
    a, fa = B.fdlb_diag(ctx)
    b, fb = B.fdlb_diag_noalloc(ctx)
    return a, fa, b, fb


def test_noalloc_diag_equals_diag_on_two_calls(P):
    B = P.B
    say("no-alloc diag: f64 300x100 reflection, 10 steps")
    p, flds, _ = fi.reflection_1024x256(lam=2.0, mach=5.0)
    p = dict(p, nx=300, ny=100)
    flds = fi.reflection_fields(300, 100, p["dx"], p["bc_state"][0], p["bc_state"][3], 29.0)
    s = P.Solver(p, precision="f64")
    s.set_state(*flds)
    s.step(10)
    a, fa, b, fb = _both(B, s.ctx)
    s.close()
    assert np.array_equal(a, b) and fa == fb and not fa, (a, b)
    assert a[0] > 0

    say("no-alloc diag: f32dev 70x19 random, 5 steps (second, smaller call)")
    st = [(1.1, 0.4, -0.1, 0.9)] * 4
    p2 = fi.problem(70, 19, 2e-3, 2e-5, 3e-5, 1.5, ("dirichlet", "outflow", "wall", "dirichlet"), st)
    s2 = P.Solver(p2, precision="f32dev")
    s2.set_state(*fi.random_fields(70, 19, seed=2))
    s2.step(5)
    a2, fa2, b2, fb2 = _both(B, s2.ctx)
    s2.close()
    assert np.array_equal(a2, b2) and fa2 == fb2, (a2, b2)
    assert not np.array_equal(a, a2)


def test_noalloc_diag_batch_and_flag(P):
    B = P.B
    say("no-alloc diag: f32 batch of 5 tubes, then a non-physical state")
    probs, _ = fi.ensemble_tubes(count=5)
    b = P.BatchSolver([q for q, _ in probs], precision="f32")
    for i, (_, fl) in enumerate(probs):
        b.set_state(i, *fl)
    b.step(7)
    x, fx, y, fy = _both(B, b.ctx)
    b.close()
    assert np.array_equal(x, y) and fx == fy and not fx
    # a state that is non-physical from the start: both report the flag
    p = fi.problem(40, 8, 1e-2, 1e-4, 2e-4, 1.0, ("periodic",) * 4)
    r, u, w, T = fi.uniform_fields(40, 8, (1.0, 0.0, 0.0, 1.0))
    T = T.copy()
    T[3, 5] = -0.5
    s = P.Solver(p, precision="f64")
    s.set_state(r, u, w, T)
    a, fa, c, fc = _both(B, s.ctx)
    s.close()
    assert fa and fc and np.array_equal(a, c)


def test_noalloc_diag_rejects_grids_beyond_its_scratch(P):
    B = P.B
    say("no-alloc diag: 4097 x 4096 float32 context (over 2^24 cells) is rejected")
    p = fi.problem(4097, 4096, 1e-3, 1e-5, 2e-5, 1.0, ("periodic",) * 4)
    s = P.Solver(p, precision="f32")
    with pytest.raises(B.FdlbError) as ei:
        B.fdlb_diag_noalloc(s.ctx)
    s.close()
    assert ei.value.status == B.FDLB_EINVAL
    assert "partial blocks" in str(ei.value)
