"""Two steps per pass (tblock = 2, float64): tiles whose cells and four cells around them lie
inside the grid take two steps per launch, the others single steps through a third buffer.
The result must be that of single steps, and so the oracle's, bit for bit: on grids with
every tile role (band tiles next to the sides, ring tiles beside them, inner two-step tiles),
every side kind, moving side segments, odd step counts, the captured graphs, and the full
benchmark grid."""
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


def run(P, prob, flds, chunks, tblock):
    s = P.Solver(prob, precision="f64", tblock=tblock)
    s.set_state(*flds)
    for c in chunks:
        s.step(c)
    f = s.get_f(allow_nonphys=True)
    kinds = [P.B.fdlb_tile_cells(s.ctx, k) for k in range(4)]
    s.close()
    return f, kinds


TX, TY = 16, 8  # two-step tile


def two_step_cells(nx, ny):
    """Cells of the tiles whose cells and four cells around them lie inside the grid."""
    cols = sum(1 for x0 in range(0, nx, TX) if x0 >= 4 and x0 + TX + 4 <= nx)
    rows = sum(1 for y0 in range(0, ny, TY) if y0 >= 4 and y0 + TY + 4 <= ny)
    return cols * rows * TX * TY


def assert_same(a, b, what):
    if not np.array_equal(a, b):
        d = int(np.count_nonzero(a != b))
        raise AssertionError(f"{what}: {d} of {a.size} values differ")


SIDES = [("dirichlet", "outflow", "wall", "dirichlet"), ("wall", "wall", "outflow", "outflow"),
         ("periodic", "periodic", "periodic", "periodic")]


@pytest.mark.parametrize("sides", SIDES)
@pytest.mark.parametrize("chunks", [(2,), (3,), (1, 10, 1), (40,)])
def test_two_step_bitwise_with_oracle(P, sides, chunks):
    say("two-step", sides, chunks)
    nx, ny = 140, 44
    st = [(1.1, 0.4, -0.1, 0.9), (1.0, 0.2, 0.05, 1.1), (1.0, 0.3, 0.0, 1.0), (0.9, 0.35, -0.2, 1.2)]
    prob = fi.problem(nx, ny, 2e-3, 2e-5, 3e-5, 1.5, sides, st)
    flds = fi.random_fields(nx, ny, seed=11)
    f2, kinds = run(P, prob, flds, chunks, 2)
    assert kinds[3] == two_step_cells(nx, ny) == 28 * 128 and sum(kinds) == nx * ny
    f1, _ = run(P, prob, flds, chunks, 1)
    assert_same(f2, f1, "two-step against single steps")
    f_ref, bad = oracle.run_f(prob, oracle.init_state(prob, flds), sum(chunks), nthreads=NTHR)
    assert bad == -1
    assert_same(f2, f_ref, "two-step against the oracle")


def test_two_step_moving_segments_and_walls(P):
    """Double Mach reflection geometry (moving top segment, wall from x = 0.08): the band's
    two single steps take the clock at t and t + dt."""
    say("two-step double mach reflection 160 x 64, 34 steps")
    prob, flds, _ = fi.double_mach(nx=160, ny=64, mach=5.0, lam=20.0)
    f2, kinds = run(P, prob, flds, (34,), 2)
    assert kinds[3] > 0
    f_ref, bad = oracle.run_f(prob, oracle.init_state(prob, flds), 34, nthreads=NTHR)
    assert bad == -1
    assert_same(f2, f_ref, "two-step DMR against the oracle")


def test_two_step_small_grid_has_only_band_tiles(P):
    say("two-step on a tube and on a grid smaller than a two-step tile's reach")
    p, flds, _ = fi.sod_tube(nx=96, ny=4)
    f2, kinds = run(P, p, flds, (9,), 2)
    assert kinds[3] == 0
    f1, _ = run(P, p, flds, (9,), 1)
    assert_same(f2, f1, "tube")


def test_two_step_benchmark_grid(P):
    say("two-step on the 8192 x 2048 Mach-20 reflection, 4 steps, against single steps")
    prob, flds, _ = fi.cfg5_reflection()
    f2, kinds = run(P, prob, flds, (4,), 2)
    assert kinds[3] == two_step_cells(prob["nx"], prob["ny"]) == (prob["nx"] - 32) * (prob["ny"] - 16)
    f1, _ = run(P, prob, flds, (4,), 1)
    assert_same(f2, f1, "benchmark grid")


def test_two_step_trials_leave_the_state(P):
    say("two-step: kernel timing, copy ceiling and autotuning leave the state")
    B = P.B
    nx, ny = 140, 44
    prob = fi.problem(nx, ny, 2e-3, 2e-5, 3e-5, 1.5, SIDES[0], [(1.0, 0.3, 0.0, 1.0)] * 4)
    flds = fi.random_fields(nx, ny, seed=3)
    s = P.Solver(prob, precision="f64", tblock=2)
    s.set_state(*flds)
    s.step(5)
    before = s.get_f()
    assert B.fdlb_time_kernel(s.ctx, 3, 4) > 0
    assert B.fdlb_time_kernel(s.ctx, -1, 4) > 0
    assert B.fdlb_copy_ceiling(s.ctx, 4) > 0
    sh, g, ms = s.autotune(trial_steps=4, groups=(4, 16))
    assert sh == 8 and ms > 0  # the 16 x 8 shape
    with pytest.raises(B.FdlbError):
        s.set_tiling(4, 16)  # the two-step tiles have one shape
    assert np.array_equal(s.get_f(), before)
    s.step(5)
    after = s.get_f()
    s.close()
    f1, _ = run(P, prob, flds, (10,), 1)
    assert_same(after, f1, "after trials")


def test_two_step_batch_equals_single_runs(P):
    """A batch of instances of uneven size (two grids with two-step tiles, a tube with none)
    with two steps per pass: each instance's moments equal its own single-step run's, bit
    for bit, after an odd number of steps (a graph of pairs and a lone single step)."""
    say("two-step batch of three uneven instances, 37 steps, against single runs")
    st = [(1.1, 0.4, -0.1, 0.9), (1.0, 0.2, 0.05, 1.1), (1.0, 0.3, 0.0, 1.0), (0.9, 0.35, -0.2, 1.2)]
    cases = [(fi.problem(140, 44, 2e-3, 2e-5, 3e-5, 1.5, SIDES[0], st), fi.random_fields(140, 44, seed=21)),
             (fi.problem(96, 40, 2e-3, 2e-5, 3e-5, 1.5, SIDES[1], st), fi.random_fields(96, 40, seed=22))]
    tube, tf, _ = fi.sod_tube(nx=96, ny=4)
    cases.append((tube, tf))
    b = P.BatchSolver([p for p, _ in cases], precision="f64", tblock=2)
    for i, (_, flds) in enumerate(cases):
        b.set_state(i, *flds)
    b.step(37)
    got = [b.moments(i) for i in range(len(cases))]
    b.close()
    for i, (prob, flds) in enumerate(cases):
        s = P.Solver(prob, precision="f64")
        s.set_state(*flds)
        s.step(37)
        ref = s.moments()
        s.close()
        for name, a, r in zip(("rho", "ux", "uy", "T"), got[i], ref):
            assert np.array_equal(a, r), (i, name, int(np.count_nonzero(a != r)))
