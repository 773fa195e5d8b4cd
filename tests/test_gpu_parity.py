"""GPU parity: the HIP path (through the C interface) against the CPU oracle on the same
seeded inputs.

Float64 mode evaluates the same formulas in the same order as the oracle without fused
multiply-adds, so the bar for it is bit-for-bit equality of all 33 distributions (which is
stronger than the 1e-12 relative tolerance of the float64 target).  Float32 mode is held
to stated L1 bounds of rho, u, T.
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


def gpu_run(P, prob, fields, nsteps, precision="f64", tile=0, chunks=None):
    s = P.Solver(prob, precision=precision, tile=tile)
    s.set_state(*fields)
    if chunks is None:
        s.step(nsteps)
    else:
        for c in chunks:
            s.step(c)
    f = s.get_f(allow_nonphys=True)
    m = s.moments(allow_nonphys=True)
    s.close()
    return f, m


def assert_bitwise(f_gpu, f_ref, what):
    if np.array_equal(f_gpu, f_ref):
        return
    d = np.abs(f_gpu - f_ref)
    rel = np.max(d / np.maximum(np.abs(f_ref), 1e-300))
    idx = np.unravel_index(np.argmax(d), d.shape)
    ndiff = int(np.count_nonzero(f_gpu != f_ref))
    raise AssertionError(f"{what}: {ndiff} of {f_ref.size} values differ; max rel {rel:.3e} at {idx}: "
                         f"gpu {f_gpu[idx]!r} oracle {f_ref[idx]!r}")


BC_COMBOS = {
    "periodic": ("periodic",) * 4,
    "reflection": ("dirichlet", "outflow", "wall", "dirichlet"),
    "walls": ("wall",) * 4,
    "tube": ("outflow", "outflow", "periodic", "periodic"),
    "mixed": ("wall", "dirichlet", "outflow", "wall"),
}


def small_case(bc_name, nx=75, ny=21, seed=0):
    st = [(1.1, 0.4, -0.1, 0.9), (0.9, -0.2, 0.3, 1.2), (1.0, 0.1, 0.2, 1.1), (1.2, 0.0, -0.3, 0.8)]
    prob = fi.problem(nx, ny, 2e-3, 2e-5, 3e-5, 1.5, BC_COMBOS[bc_name], st)
    return prob, fi.random_fields(nx, ny, seed=seed)


@pytest.mark.parametrize("bc_name", list(BC_COMBOS))
def test_f64_bitwise_small_grid(P, bc_name):
    say("f64 bitwise", bc_name, "75x21, 12 steps")
    prob, flds = small_case(bc_name)
    f_gpu, m_gpu = gpu_run(P, prob, flds, 12)
    f_ref, bad = oracle.run_f(prob, oracle.init_state(prob, flds), 12, nthreads=NTHR)
    assert bad == -1
    assert_bitwise(f_gpu, f_ref, bc_name)
    m_ref = oracle.fields(prob, f_ref)
    for a, b in zip(m_gpu, m_ref):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape", range(1, 8))
def test_f64_bitwise_every_tile_shape(P, shape):
    say("f64 bitwise tile shape", shape)
    prob, flds = small_case("reflection", nx=131, ny=37, seed=shape)
    f_gpu, _ = gpu_run(P, prob, flds, 6, tile=shape)
    f_ref, _ = oracle.run_f(prob, oracle.init_state(prob, flds), 6, nthreads=NTHR)
    assert_bitwise(f_gpu, f_ref, f"shape {shape}")


@pytest.mark.parametrize("nx,ny,bc", [(1, 1, "periodic"), (3, 2, "periodic"), (2, 5, "walls"), (7, 1, "tube"),
                                      (5, 3, "reflection"), (2, 2, "mixed")])
def test_f64_bitwise_grids_smaller_than_a_tile(P, nx, ny, bc):
    say("f64 tiny grid", nx, ny, bc)
    prob, flds = small_case(bc, nx=nx, ny=ny, seed=nx * 7 + ny)
    f_gpu, _ = gpu_run(P, prob, flds, 5)
    f_ref, _ = oracle.run_f(prob, oracle.init_state(prob, flds), 5, nthreads=1)
    assert_bitwise(f_gpu, f_ref, f"{nx}x{ny}")


def test_f64_zero_steps_is_the_equilibrium(P):
    say("f64 zero steps")
    prob, flds = small_case("reflection", nx=40, ny=9)
    f_gpu, _ = gpu_run(P, prob, flds, 0)
    assert_bitwise(f_gpu, oracle.init_state(prob, flds), "init")


def test_graph_replay_equals_single_launches(P):
    say("graph replay vs launches")
    prob, flds = small_case("reflection", nx=64, ny=16)
    a, _ = gpu_run(P, prob, flds, 70)
    b, _ = gpu_run(P, prob, flds, 70, chunks=[1] * 70)
    c, _ = gpu_run(P, prob, flds, 70, chunks=[33, 5, 32])
    assert np.array_equal(a, b) and np.array_equal(a, c)


@pytest.mark.parametrize("fork,edge_tile", [("0", "0"), ("1", "0"), ("1", "7"), ("1", "5"), ("0", "2")])
def test_graph_branch_and_edge_pieces_bitwise(P, monkeypatch, fork, edge_tile):
    """Captured steps with the edge tiles as a parallel branch or serial (FDLB_GRAPH_FORK),
    and edge tiles launched whole or cut into 32 x 4, 16 x 4 or 64 x 4 pieces
    (FDLB_EDGE_TILE): every variant equals the oracle bit for bit, through the graphs (96
    steps) and for a batch of uneven tubes."""
    monkeypatch.setenv("FDLB_GRAPH_FORK", fork)
    monkeypatch.setenv("FDLB_EDGE_TILE", edge_tile)
    say("graph branch", fork, "edge tile", edge_tile, "reflection 200x72, 96 steps")
    prob, flds = small_case("reflection", nx=200, ny=72)
    f_gpu, _ = gpu_run(P, prob, flds, 96)
    f_ref, _ = oracle.run_f(prob, oracle.init_state(prob, flds), 96, nthreads=NTHR)
    assert_bitwise(f_gpu, f_ref, f"fork {fork} edge tile {edge_tile}")
    probs = [fi.problem(nx, 4, 2e-3, 2e-5, 3e-5, 1.5, BC_COMBOS["tube"]) for nx in (150, 67, 301)]
    fields = [fi.random_fields(p["nx"], 4, seed=i) for i, p in enumerate(probs)]
    b = P.BatchSolver(probs, precision="f64")
    for i, fl in enumerate(fields):
        b.set_state(i, *fl)
    b.step(64)
    for i, (p, fl) in enumerate(zip(probs, fields)):
        m = b.moments(i)
        f_ref, bad = oracle.run_f(p, oracle.init_state(p, fl), 64)
        assert bad == -1, i
        for a, r in zip(m, oracle.fields(p, f_ref)):
            assert np.array_equal(a, r), f"batch instance {i}"
    b.close()


def test_checkpoint_resume_is_bitwise(P):
    say("checkpoint resume")
    prob, flds = small_case("mixed", nx=50, ny=30)
    s = P.Solver(prob)
    s.set_state(*flds)
    s.step(20)
    ck = s.get_f()
    s.step(20)
    full = s.get_f()
    s2 = P.Solver(prob)
    s2.set_f(ck)
    s2.step(20)
    assert np.array_equal(s2.get_f(), full)
    s.close()
    s2.close()


def test_sod_400x4_full_run_bitwise(P):
    say("sod 400x4 1000 steps")
    prob, flds, nsteps = fi.sod_tube()
    f_gpu, m_gpu = gpu_run(P, prob, flds, nsteps)
    f_ref, bad = oracle.run_f(prob, oracle.init_state(prob, flds), nsteps, nthreads=NTHR)
    assert bad == -1
    assert_bitwise(f_gpu, f_ref, "sod")


def test_uniform_mach20_stays_bitwise_uniform(P):
    """The Mach-20 inflow state is linearly unstable without the switch (Sec. 4, Fig. 6);
    it survives only because every cell does the same operations.  10^4 steps on several
    tiles, periodic, compared with the oracle."""
    say("uniform mach 20, 64x16, 10000 steps")
    prob = fi.problem(64, 16, 2.5e-4, 1e-6, 2e-6, 2.0, ("periodic",) * 4)
    flds = fi.uniform_fields(64, 16, fi.REFL_PRE)
    f_gpu, _ = gpu_run(P, prob, flds, 10000)
    for q in range(33):
        assert np.all(f_gpu[q] == f_gpu[q, 0, 0])
    f_ref, _ = oracle.run_f(prob, oracle.init_state(prob, flds), 10000, nthreads=NTHR)
    assert_bitwise(f_gpu, f_ref, "uniform")


def test_reflection_1024x256_freestream_mach5_bitwise(P):
    """The 29-degree reflection at freestream Mach 5 (a reading that stays physical for the
    full 40000 steps), 40 steps on the full grid."""
    say("reflection 1024x256 mach 5, 40 steps")
    prob, flds, _ = fi.reflection_1024x256(lam=2.0, mach=5.0)
    f_gpu, _ = gpu_run(P, prob, flds, 40)
    f_ref, bad = oracle.run_f(prob, oracle.init_state(prob, flds), 40, nthreads=NTHR)
    assert bad == -1
    assert_bitwise(f_gpu, f_ref, "reflection m5")


def test_reflection_1024x256_normal_mach10_bitwise_while_finite(P):
    """The literal reading (shock normal Mach 10) turns non-physical after the first step in
    the oracle as in the GPU path (T < 0 below the incident shock); the two agree bit for bit
    while every value is finite."""
    say("reflection 1024x256 normal mach 10, 3 steps")
    prob, flds, _ = fi.reflection_1024x256(lam=2.0, mach_n=10.0)
    f_gpu, _ = gpu_run(P, prob, flds, 3)
    f_ref, bad = oracle.run_f(prob, oracle.init_state(prob, flds), 3, nthreads=NTHR)
    assert bad == 2
    assert np.all(np.isfinite(f_ref))
    assert_bitwise(f_gpu, f_ref, "reflection mn10")


def test_reflection_8192x2048_full_grid_bitwise(P):
    """The benchmark grid (8192 x 2048, Mach 5 reading) for a few steps, every value."""
    say("reflection 8192x2048 mach 5, 3 steps")
    prob, flds, _ = fi.reflection_8192x2048(mach=5.0)
    f_gpu, _ = gpu_run(P, prob, flds, 3)
    f_ref, bad = oracle.run_f(prob, oracle.init_state(prob, flds), 3, nthreads=NTHR)
    assert bad == -1
    assert_bitwise(f_gpu, f_ref, "reflection 8192x2048")


def test_nonphysical_state_is_reported(P):
    say("non-physical flag")
    prob, flds = small_case("periodic", nx=20, ny=8)
    r = flds[0].copy()
    r[3, 4] = -0.5
    s = P.Solver(prob)
    s.set_state(r, *flds[1:])
    with pytest.raises(P.FdlbError) as e:
        s.moments()
    assert e.value.status == P.FDLB_ENONPHYS
    _, flag = s.diag()
    assert flag
    s.close()


def test_diag_totals_match_oracle_moments(P):
    say("diag totals")
    prob, flds = small_case("periodic", nx=64, ny=24)
    s = P.Solver(prob)
    s.set_state(*flds)
    s.step(10)
    sums, flag = s.diag()
    assert not flag
    f_ref, _ = oracle.run_f(prob, oracle.init_state(prob, flds), 10, nthreads=NTHR)
    vx, vy = oracle.velocities(prob["v"])
    e = 0.5 * (vx * vx + vy * vy)
    want = [f_ref.sum(), (vx[:, None, None] * f_ref).sum(), (vy[:, None, None] * f_ref).sum(),
            (e[:, None, None] * f_ref).sum()]
    np.testing.assert_allclose(sums, want, rtol=1e-12, atol=1e-12)
    s.close()


def test_f32_sod_l1_bounds(P):
    """Float32 storage on a well-conditioned tube (sum |f| / n ~ 1): stated L1 bounds of
    rho, u, T against the float64 oracle after 1000 steps."""
    say("f32 sod")
    prob, flds, nsteps = fi.sod_tube()
    _, m32 = gpu_run(P, prob, flds, nsteps, precision="f32")
    m64, _ = oracle.run_state(prob, flds, nsteps, nthreads=NTHR)
    l1 = [np.mean(np.abs(a - b)) / np.mean(np.abs(b) + 1e-300) for a, b in zip(m32, m64)]
    assert l1[0] < 1e-5 and l1[3] < 1e-5, l1
    assert np.mean(np.abs(m32[1] - m64[1])) < 1e-5


def test_batch_equals_single_runs(P):
    say("batch vs single")
    cases = [small_case("tube", nx=nx, ny=4, seed=nx) for nx in (300, 77, 129)]
    b = P.BatchSolver([c[0] for c in cases], precision="f64")
    for i, (prob, flds) in enumerate(cases):
        b.set_state(i, *flds)
    b.step(40)
    for i, (prob, flds) in enumerate(cases):
        mb = b.moments(i)
        f_ref, _ = oracle.run_f(prob, oracle.init_state(prob, flds), 40, nthreads=NTHR)
        m_ref = oracle.fields(prob, f_ref)
        for x, y in zip(mb, m_ref):
            assert np.array_equal(x, y), i
    b.close()


@pytest.mark.parametrize("precision", ["f64", "f32", "f32dev"])
def test_copy_ceiling_and_kernel_timing_leave_the_state(P, precision):
    """The bandwidth reference (a plain copy of the stored planes) and the kernel timing
    write only the other half: the state and the following steps are unchanged."""
    say("copy ceiling", precision)
    prob, flds = small_case("reflection", nx=300, ny=70)
    a = P.Solver(prob, precision=precision)
    a.set_state(*flds)
    a.step(5)
    f0 = a.get_f()
    assert P.B.fdlb_copy_ceiling(a.ctx, 3) > 0 and P.B.fdlb_time_kernel(a.ctx, -1, 2) > 0
    f1 = a.get_f()
    same = (lambda x, y: all(np.array_equal(u, v) for u, v in zip(x, y))) if precision == "f32dev" \
        else np.array_equal
    assert same(f0, f1)
    a.step(7)
    b = P.Solver(prob, precision=precision)
    b.set_state(*flds)
    b.step(12)
    assert same(a.get_f(), b.get_f())
    a.close()
    b.close()


def test_autotune_leaves_state_and_results_unchanged(P):
    """The autotuner's trial steps never advance the state, and every tiling gives the same
    bits."""
    say("autotune")
    prob, flds = small_case("reflection", nx=300, ny=70)
    a = P.Solver(prob)
    a.set_state(*flds)
    f0 = a.get_f()
    sh, g, ms = a.autotune(trial_steps=2, shape_ids=(1, 3, 4), groups=(1, 8))
    assert ms > 0 and sh in (1, 3, 4) and g in (1, 8)
    assert np.array_equal(a.get_f(), f0)
    a.step(25)
    b = P.Solver(prob)
    b.set_state(*flds)
    b.set_tiling(2, 3)
    b.step(25)
    assert np.array_equal(a.get_f(), b.get_f())
    a.close()
    b.close()


def test_colella_tau_dt_full_run_bitwise(P):
    """Colella's explosion problem at 4000 x 4, the full 20000 steps with tau = dt (the
    literal tau = 2 dt goes non-physical; both readings are compared while finite)."""
    say("colella tau=dt 4000x4 20000 steps")
    prob, flds, nsteps = fi.colella_tube(tau=1e-6)
    f_gpu, _ = gpu_run(P, prob, flds, nsteps)
    f_ref, bad = oracle.run_f(prob, oracle.init_state(prob, flds), nsteps, nthreads=NTHR)
    assert bad == 1  # the first step's dispersion kick leaves T < 0 in one cell; it recovers
    assert np.all(np.isfinite(f_ref))
    assert_bitwise(f_gpu, f_ref, "colella tau=dt")


def test_colella_literal_tau_bitwise_while_finite(P):
    say("colella tau=2dt 4000x4 300 steps")
    prob, flds, _ = fi.colella_tube()
    f_gpu, _ = gpu_run(P, prob, flds, 300)
    f_ref, _ = oracle.run_f(prob, oracle.init_state(prob, flds), 300, nthreads=NTHR)
    assert np.all(np.isfinite(f_ref))
    assert_bitwise(f_gpu, f_ref, "colella tau=2dt")


def test_ensemble_all_256_tubes_bitwise(P):
    """The batched ensemble (256 tubes of 256..4096 cells, one launch per step), every
    instance against its own oracle run."""
    say("ensemble 256 tubes, 20 steps")
    probs, _ = fi.ensemble_tubes()
    b = P.BatchSolver([p for p, _ in probs], precision="f64")
    for i, (p, flds) in enumerate(probs):
        b.set_state(i, *flds)
    b.step(20)
    for i, (p, flds) in enumerate(probs):
        mb = b.moments(i)
        f_ref, bad = oracle.run_f(p, oracle.init_state(p, flds), 20, nthreads=NTHR)
        assert bad == -1, i
        for x, y in zip(mb, oracle.fields(p, f_ref)):
            assert np.array_equal(x, y), i
    b.close()


def test_ensemble_f32_l1_bounds(P):
    """Float32 ensemble after 500 steps against float64 oracle runs of a few instances
    (smallest and largest grid, highest pressure ratio): L1 of rho, T below 1e-5, of u
    below 1e-4 (relative to the largest |u|)."""
    say("ensemble f32, 500 steps")
    probs, _ = fi.ensemble_tubes()
    b = P.BatchSolver([p for p, _ in probs], precision="f32")
    for i, (p, flds) in enumerate(probs):
        b.set_state(i, *flds)
    b.step(500)
    draws = fi.ensemble_draws()
    pick = {min(range(256), key=lambda i: draws[i][0]), max(range(256), key=lambda i: draws[i][0]),
            max(range(256), key=lambda i: draws[i][1])}
    for i in sorted(pick):
        p, flds = probs[i]
        m32 = b.moments(i)
        m64, bad = oracle.run_state(p, flds, 500, nthreads=NTHR)
        assert bad == -1
        l1 = [np.mean(np.abs(a - c)) for a, c in zip(m32, m64)]
        assert l1[0] / np.mean(m64[0]) < 1e-5 and l1[3] / np.mean(m64[3]) < 1e-5, (i, l1)
        assert l1[1] / max(np.max(np.abs(m64[1])), 1e-30) < 1e-4, (i, l1)
    b.close()
