"""Host-side behaviour of the C interface around trial launches and batches, on the GPU:
timing and autotuning leave the state and the sticky non-physical flag as they were, and a
batch refuses to re-set one instance once it has stepped (its instances share one step
clock and one flag)."""
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


def _mach20_uniform_start():
    """The Mach-20 inflow everywhere under the printed post-shock top state (Sec. 5.2.1,
    300 x 100, dx = 3e-3, dt = tau = 1e-5): physical after one step (T = 0.18 two rows
    under the top), non-physical after the second."""
    pre, post = fi.REFL_PRE, fi.REFL_POST_PRINTED
    p = fi.problem(300, 100, 3e-3, 1e-5, 1e-5, 2.0, ("dirichlet", "outflow", "wall", "dirichlet"),
                   (pre, pre, pre, post))
    return p, fi.uniform_fields(300, 100, pre)


@pytest.mark.parametrize("what", ["time_kernel", "autotune"])
def test_trial_launches_keep_the_flag(P, what):
    say("trial launches keep the flag:", what)
    B = P.B
    p, flds = _mach20_uniform_start()
    s = P.Solver(p, precision="f64")
    s.set_state(*flds)
    s.step(1)
    _, bad = s.diag()
    assert not bad
    f_before = s.get_f()
    if what == "time_kernel":
        B.fdlb_time_kernel(s.ctx, -1, 3)
        B.fdlb_time_kernel(s.ctx, 0, 3)
    else:
        s.autotune(trial_steps=2, shape_ids=(1, 4), groups=(8,))
    _, bad = s.diag()
    assert not bad, "a trial step raised the flag of a state that never took it"
    assert np.array_equal(s.get_f(), f_before)
    s.step(1)  # the real second step is non-physical
    _, bad = s.diag()
    s.close()
    assert bad


def test_batch_set_state_after_stepping_is_refused(P):
    say("batch set_state after stepping")
    B = P.B
    probs, _ = fi.ensemble_tubes(count=3)
    b = P.BatchSolver([q for q, _ in probs], precision="f64")
    for i, (_, fl) in enumerate(probs):
        b.set_state(i, *fl)
    b.set_state(1, *probs[1][1])  # before stepping: allowed
    b.step(4)
    with pytest.raises(B.FdlbError) as ei:
        b.set_state(1, *probs[1][1])
    assert ei.value.status == B.FDLB_ESTATE
    b.step(1)
    assert B.fdlb_steps_done(b.ctx) == 5
    b.close()
