"""Benchmark of the FDLB hot path on one MI355X.

Headline workload: the paper's Mach-20 steady regular reflection (Sec. 5.2.1 inflow
(1, 20, 0, 0.5), 30-degree incident shock, printed post-shock state on the top side,
reflecting wall at the bottom, outflow on the right) on 8192 x 2048 cells, dx = dy = 2.5e-4,
dt = tau = 1e-6, artificial-viscosity amplitude lambda = 40, incident shock smoothed over two
cells at t = 0.  (With tau = 2 dt, lambda <= 30 or a sharp start the printed scheme turns
non-physical within 1000-4000 steps on this grid.)  A step is one launch per tile kind that
advances all 33 distributions of every cell by Eq. (dis_eq1); `value` is the float64 rate
over the timed steps, with the inputs resident in HBM.

Reported in the one JSON line:
  - `value`, `roofline` (the float64 interior kernel timed alone with HIP events on the
    context's stream, algorithmic bytes 528 per cell-update, against 8 TB/s; counter
    traffic from the committed profile when it matches the kernel source; a plain copy of
    the same planes over the same tiles as the practical ceiling), `graph_replay_64` (64
    steps through the captured 32-step graphs, whatever --steps is);
  - `f32`, `f32dev`: the two float32 storages on the same workload (rate, speed-up,
    relative L1 / Linf of rho, u, T against float64 after the timed steps);
  - `configs`: one block per configuration with its own full step count: Sod 400 x 4,
    Colella 4000 x 4 (with the L1 against the exact solution), the 1024 x 256 reflection,
    the 256-tube ensemble (named pressure-ratio range and the physical one, autotuned
    against default tiling), and the 8192 x 2048 reflection's accuracy at 10000 steps;
    plus float32 against float64 on the same grid with Mach-5 and Mach-10 inflows, where the
    float32 storages can hold the flow;
  - `two_step`: the same workload with two steps per pass (tblock = 2); `vn_sweep`: the
    stability analysis of Sec. 4 on the GPU (double-double spectral radii);
  - `cpu_baseline`: the float64 oracle on a bounded slice of the headline grid, on one
    thread and on the host threads the job may use, and one matrix of the mpmath stability
    tool.
"""
import argparse
import hashlib
import json
import os
import platform
import re
import subprocess
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# compulsory read + write per cell-update: the 33 planes, plus the four float64 moments of
# the deviation storage
ALG_BYTES = {"f64": 2 * 33 * 8, "f32": 2 * 33 * 4, "f32dev": 2 * (33 * 4 + 4 * 8)}
KERNEL_SRC = os.path.join(ROOT, "paper_0801_4169_amd", "csrc", "fdlb_kernels.hip")
# counter summaries of the interior kernel per storage (rocprofv3 FETCH_SIZE / WRITE_SIZE)
COUNTERS = {pr: os.path.join(ROOT, "profiles", f"step_interior_{pr}_reflection_8192x2048_counters.md")
            for pr in ("f64", "f32", "f32dev")}
COUNTERS["step2"] = os.path.join(ROOT, "profiles", "step2_f64_reflection_8192x2048_counters.md")
COLELLA_EXACT = os.path.join(ROOT, "tests", "golden", "colella_exact_j4m.json")
STORAGES = ("f64", "f32", "f32dev")


def say(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--nx", type=int, default=8192)
    ap.add_argument("--ny", type=int, default=2048)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--configs", default="1,2,3,4,5",
                    help="configuration blocks to run (comma list of 1..5; empty: none)")
    ap.add_argument("--no-extras", action="store_true", help="skip the two-step and stability-sweep legs")
    ap.add_argument("--cpu-steps", type=int, default=160, help="oracle steps of the CPU baseline slice (0: skip)")
    ap.add_argument("--cpu-rows", type=int, default=128, help="rows of the CPU baseline slice")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB (calibrates the HBM "
                         "byte counters of a profiler run against a kernel of known traffic)")
    return ap.parse_args()


def src_hash():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def committed_traffic(precision="f64"):
    """HBM bytes per interior-kernel launch of a storage from its committed counter summary,
    if it was taken on the current kernel source."""
    path = COUNTERS[precision]
    if not os.path.exists(path):
        return None
    text = open(path).read()
    h = re.search(r"kernel source sha256\[:16\]: ([0-9a-f]+)", text)
    b = re.search(r"traffic bytes per launch: ([0-9.eE+]+)", text)
    if not h or not b or h.group(1) != src_hash():
        return None
    return float(b.group(1))


def l1_rel(a, b):
    import numpy as np
    return float(np.sum(np.abs(a - b)) / max(np.sum(np.abs(b)), 1e-300))


def linf_rel(a, b):
    import numpy as np
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def errors(m, ref):
    """Relative L1 and Linf of (rho, u, T) of moments m against ref; u is the velocity
    vector (both components over the largest reference component)."""
    import numpy as np
    out = {}
    for k, i in (("rho", 0), ("T", 3)):
        out[k] = {"l1": l1_rel(m[i], ref[i]), "linf": linf_rel(m[i], ref[i])}
    du = np.abs(m[1] - ref[1]) + np.abs(m[2] - ref[2])
    su = np.abs(ref[1]) + np.abs(ref[2])
    out["u"] = {"l1": float(du.sum() / max(su.sum(), 1e-300)), "linf": float(du.max() / max(su.max(), 1e-300))}
    return out


def physical(m):
    import numpy as np
    return bool(np.all(np.isfinite(m[3])) and np.all(m[0] > 0) and np.all(m[3] > 0))


def events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def timed_steps(solver, n):
    """ms of n steps of a solver, torch events on the solver's stream (torch's current one)."""
    import torch
    torch.cuda.synchronize()
    e0, e1 = events()
    e0.record()
    solver.step(n)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def release(solver):
    import torch
    solver.close()
    del solver
    torch.cuda.empty_cache()


def headline_run(P, prob, fields, precision, steps, warmup, tile, graph_leg):
    s = P.Solver(prob, precision=precision, tile=tile)
    s.set_state(*fields)
    s.step(warmup)
    ms = timed_steps(s, steps)
    out = dict(ms=ms)
    m = s.moments(allow_nonphys=True)
    _, flag = s.diag()
    # the dominant kernel (interior tiles) alone, HIP events on the same stream
    out["k_ms"] = P.B.fdlb_time_kernel(s.ctx, 0, 50)
    out["k_cells"] = P.B.fdlb_tile_cells(s.ctx, 0)
    # the practical ceiling: a plain copy of the stored planes over the same tiles
    out["copy_ms"] = P.B.fdlb_copy_ceiling(s.ctx, 50)
    out["tiling"] = list(s.tiling)
    if graph_leg:
        out["graph64_ms"] = timed_steps(s, 64)
    release(s)
    out.update(moments=m, flag=flag)
    return out


def fixed_run(P, prob, fields, precision, steps, check=0, tile=0):
    """A run of `steps` steps: (ms, moments at the end, first check point where the flag
    was up or None, tiling).  With `check` > 0 the run is cut into pieces of that many steps
    and the flag is read after each; the time is the sum of the pieces' step time alone."""
    s = P.Solver(prob, precision=precision, tile=tile)
    s.set_state(*fields)
    s.step(0)
    first = None
    if check <= 0:
        ms = timed_steps(s, steps)
    else:
        ms, done = 0.0, 0
        while done < steps:
            k = min(check, steps - done)
            ms += timed_steps(s, k)
            done += k
            if first is None and s.diag()[1]:
                first = done
    m = s.moments(allow_nonphys=True)
    if first is None and s.diag()[1]:
        first = steps
    tiling = list(s.tiling)
    release(s)
    return ms, m, first, tiling


def rate_block(cells, steps, ms, precision):
    sec = ms / 1e3
    return {"Mcell_updates_per_s": cells * steps / sec / 1e6, "us_per_step": ms * 1e3 / steps,
            "hbm_frac": ALG_BYTES[precision] * cells * steps / sec / 1e9 / HBM_PEAK_GBS}


def storages_on(P, prob, fields, steps, check=0, extra=None):
    """Every storage on one workload for `steps` steps: rate, physical or not (first flagged
    check point) and errors against float64."""
    cells = prob["nx"] * prob["ny"]
    res, mom = {}, {}
    for pr in STORAGES:
        say(f"{prob['name']}: {pr}, {steps} steps")
        ms, m, first, tiling = fixed_run(P, prob, fields, pr, steps, check)
        mom[pr] = m
        res[pr] = dict(rate_block(cells, steps, ms, pr), physical=physical(m), first_flag_by=first, tiling=tiling)
    for pr in ("f32", "f32dev"):
        if res[pr]["physical"] and res["f64"]["physical"]:
            res[pr]["vs_f64"] = errors(mom[pr], mom["f64"])
        res[pr]["speedup_vs_f64"] = res[pr]["Mcell_updates_per_s"] / res["f64"]["Mcell_updates_per_s"]
    if extra:
        extra(res, mom)
    return res, mom


def cfg1(P, fi):
    prob, fields, steps = fi.sod_tube()
    res, _ = storages_on(P, prob, fields, steps)
    return {"workload": prob["name"], "steps": steps, "dt": prob["dt"], "tau": prob["tau"], "lambda": prob["lam"],
            "note": "cache-resident and launch-bound: us_per_step is the figure; float64 is bit-identical to "
                    "the oracle (tests/test_gpu_parity.py)", **res}


def cfg2(P, fi):
    import numpy as np
    prob, fields, steps = fi.colella_tube(tau=1e-6)
    exact = json.load(open(COLELLA_EXACT))
    j = np.array(exact["j"])
    smooth = np.array(exact["smooth"], dtype=bool)
    ref = {k: np.array(exact[k]) for k in ("rho", "u", "T")}

    def vs_exact(res, mom):
        for pr in STORAGES:
            m = mom[pr]
            if not res[pr]["physical"]:
                continue
            row = {"rho": m[0][0, j], "u": m[1][0, j], "T": m[3][0, j]}
            ent = {}
            for k in ("rho", "u", "T"):
                d = np.abs(row[k] - ref[k])
                scale = np.abs(ref[k]) if k != "u" else np.full_like(ref[k], np.max(np.abs(ref[k])))
                ent[k] = {"l1_all": float(d.sum() / scale.sum()),
                          "l1_smooth": float(d[smooth].sum() / scale[smooth].sum())}
            res[pr]["vs_exact_j4m"] = ent

    res, _ = storages_on(P, prob, fields, steps, check=1000, extra=vs_exact)
    literal = fi.colella_tube()[0]
    say("colella: literal tau = 2 dt in float64")
    _, lm_, first, _ = fixed_run(P, literal, fields, "f64", steps, check=500)
    return {"workload": prob["name"] + "_tau_eq_dt", "steps": steps, "dt": prob["dt"], "tau": prob["tau"],
            "lambda": prob["lam"],
            "note": "tau = dt: at the specified tau = 2 dt the T = 1000 state is linearly unstable; L1 against the "
                    "exact gamma = 2 solution at the cells j = 4m, over all of them and over those 0.02 away from "
                    "every wave and both ends (the shock leaves the tube at t = 0.0197)",
            "literal_tau_2dt_f64": {"first_flag_by": first, "physical_at_end": physical(lm_)}, **res}


def cfg3(P, fi):
    import numpy as np
    prob, fields, steps = fi.cfg3_reflection()

    def floor(res, mom):
        rng = np.random.default_rng(1)
        pert = (fields[0] * (1.0 + 1e-13 * rng.standard_normal(fields[0].shape)),) + tuple(fields[1:])
        _, m, _, _ = fixed_run(P, prob, pert, "f64", steps)
        res["f64_with_1e-13_noise_vs_f64"] = errors(m, mom["f64"])

    res, _ = storages_on(P, prob, fields, steps, check=10000, extra=floor)
    return {"workload": prob["name"], "steps": steps, "dt": prob["dt"], "tau": prob["tau"], "lambda": prob["lam"],
            "start": "incident shock smoothed over 2 cells", **res}


def cfg4(P, fi):
    """The 256-tube ensemble: the named pressure-ratio range (log-uniform in [10, 1e5]),
    how many of its instances stay physical in float64 (bit-identical to the oracle), and the
    range [10, 100] where all do, in every storage, autotuned against default tiling."""
    import numpy as np
    import torch
    out = {"workload": "ensemble_256_tubes_seed0", "steps": 5000}
    probs, steps = fi.ensemble_tubes(log_rp_max=5.0)
    say("ensemble, pressure ratio up to 1e5: float64 with per-instance checks")
    b = P.BatchSolver([p for p, _ in probs], precision="f64")
    for i, (p, flds) in enumerate(probs):
        b.set_state(i, *flds)
    ever_bad = np.zeros(len(probs), dtype=bool)
    for _ in range(10):
        b.step(steps // 10)
        for i in range(len(probs)):
            if not physical(b.moments(i, allow_nonphys=True)):
                ever_bad[i] = True
    end_ok = np.array([physical(b.moments(i, allow_nonphys=True)) for i in range(len(probs))])
    b.close()
    rp = np.array([r for _, r, _ in fi.ensemble_draws(log_rp_max=5.0)])
    out["range_10_to_1e5_f64"] = {
        "instances": len(probs), "physical_throughout": int((~ever_bad).sum()),
        "transient_then_physical": int((ever_bad & end_ok).sum()), "non_physical_at_end": int((~end_ok).sum()),
        "largest_ratio_physical_throughout": float(rp[~ever_bad].max()) if (~ever_bad).any() else None,
        "smallest_ratio_non_physical_at_end": float(rp[~end_ok].min()) if (~end_ok).any() else None,
        "check": "moments of every instance every 500 steps"}

    probs, steps = fi.ensemble_tubes()
    cells = sum(p["nx"] * p["ny"] for p, _ in probs)
    mom = {}
    rng_out = {"pressure_ratio": "log-uniform [10, 100]", "cells": cells}
    cache = os.environ.get("FDLB_AUTOTUNE_CACHE",
                           os.path.join(tempfile.gettempdir(), "fdlb_autotune_cache.json"))
    for pr in STORAGES:
        b = P.BatchSolver([p for p, _ in probs], precision=pr)
        for i, (p, flds) in enumerate(probs):
            b.set_state(i, *flds)
        default_tiling = list(b.tiling)
        say(f"ensemble [10, 100]: {pr} default tiling {default_tiling}, {steps} steps")
        ms_default = timed_steps(b, steps)
        # results do not depend on the tiling: the accuracy comes from this run
        mom[pr] = [b.moments(i, allow_nonphys=True) for i in range(len(probs))]
        # autotuner (its trial steps leave the state as it is), then the same steps again
        sh, g, _ = b.autotune(trial_steps=20, cache=cache)
        ms_tuned = timed_steps(b, steps)
        rng_out[pr] = dict(rate_block(cells, steps, ms_tuned, pr), tiling_autotuned=[sh, g],
                           tiling_default=default_tiling, us_per_step_default_tiling=ms_default * 1e3 / steps,
                           Mcell_updates_per_s_default_tiling=cells * steps / (ms_default / 1e3) / 1e6,
                           instances_physical_at_end=sum(physical(m) for m in mom[pr]))
        b.close()
        torch.cuda.empty_cache()
    for pr in ("f32", "f32dev"):
        l1 = np.array([[l1_rel(a[k], r[k]) for k in (0, 3)] for a, r in zip(mom[pr], mom["f64"])])
        rng_out[pr]["l1_vs_f64_rho_T_median"] = [float(x) for x in np.median(l1, axis=0)]
        rng_out[pr]["l1_vs_f64_rho_T_max"] = [float(x) for x in np.max(l1, axis=0)]
        rng_out[pr]["speedup_vs_f64"] = rng_out[pr]["Mcell_updates_per_s"] / rng_out["f64"]["Mcell_updates_per_s"]
    out["range_10_to_100"] = rng_out
    return out


def cfg5_accuracy(P, fi, prob, fields, head, steps_done):
    """Errors of the float32 storages against float64 after the full 10000 steps (reusing
    the headline runs when they were at least that long), beside the float64 sensitivity
    floor."""
    import numpy as np
    steps = 10000
    if steps_done >= steps:
        steps = steps_done
        mom = {pr: head[pr]["moments"] for pr in head}
    else:
        mom = {}
        for pr in STORAGES:
            say(f"cfg5 accuracy: {pr}, {steps} steps")
            mom[pr] = fixed_run(P, prob, fields, pr, steps)[1]
    out = {"workload": prob["name"], "steps": steps}
    for pr in STORAGES:
        out[pr] = {"physical": physical(mom[pr])}
    for pr in ("f32", "f32dev"):
        if physical(mom[pr]) and physical(mom["f64"]):
            out[pr]["vs_f64"] = errors(mom[pr], mom["f64"])
    say("cfg5 accuracy: float64 with 1e-13 noise in the initial density (sensitivity floor)")
    rng = np.random.default_rng(1)
    pert = (fields[0] * (1.0 + 1e-13 * rng.standard_normal(fields[0].shape)),) + tuple(fields[1:])
    m = fixed_run(P, prob, pert, "f64", steps)[1]
    out["f64_with_1e-13_noise_vs_f64"] = errors(m, mom["f64"]) if physical(m) else "non-physical"
    return out


def accuracy_blocks(P, fi, nx, ny, steps=2000):
    """Float32 against float64 where float32 storage can hold the flow (the deviation
    storage cannot hold a Mach-20 shock: its float32 g there is as large as the cancellation
    in the equilibrium).  Same grid, sides and dt as the headline: freestream Mach 5 with
    lambda = 2 (float64 itself does not amplify rounding there), and freestream Mach 10 with
    lambda = 20 at the specified tau = 2 dt; beside each, what a 1e-13 perturbation of the
    initial density does to float64."""
    import numpy as np
    out = {}
    for name, (mach, lam) in (("accuracy_mach5", (5.0, 2.0)), ("accuracy_mach10", (10.0, 20.0))):
        prob, fields, _ = fi.reflection_8192x2048(lam=lam, nx=nx, ny=ny, mach=mach, tau=2e-6,
                                                  width=fi.SMOOTH_WIDTH)
        ent = {"workload": prob["name"], "lambda": lam, "tau": prob["tau"], "steps": steps}
        mom = {}
        for pr in STORAGES:
            say(f"{name}: {pr}, {steps} steps")
            ms, mom[pr], first, _ = fixed_run(P, prob, fields, pr, steps)
            ent[pr] = dict(rate_block(nx * ny, steps, ms, pr), physical=physical(mom[pr]))
        rng = np.random.default_rng(1)
        pert = (fields[0] * (1.0 + 1e-13 * rng.standard_normal(fields[0].shape)),) + tuple(fields[1:])
        say(f"{name}: float64 with 1e-13 noise")
        m = fixed_run(P, prob, pert, "f64", steps)[1]
        ent["f64_with_1e-13_noise_vs_f64"] = errors(m, mom["f64"])
        for pr in ("f32", "f32dev"):
            if ent[pr]["physical"]:
                ent[pr]["vs_f64"] = errors(mom[pr], mom["f64"])
            ent[pr]["speedup_vs_f64"] = ent[pr]["Mcell_updates_per_s"] / ent["f64"]["Mcell_updates_per_s"]
        out[name] = ent
    return out


def two_step(P, prob, fields, single):
    """The headline workload with two steps per pass (tblock = 2): float64 interior tiles
    take two steps per launch with the intermediate step in LDS (bit-identical to single
    steps).  Rate over 64 steps through the captured graphs, and the two-step kernel alone."""
    say("two steps per pass: float64, 64 steps")
    s = P.Solver(prob, precision="f64", tblock=2)
    s.set_state(*fields)
    s.step(8)
    ms = timed_steps(s, 64)
    k_ms = P.B.fdlb_time_kernel(s.ctx, 3, 20)
    k_cells = P.B.fdlb_tile_cells(s.ctx, 3)
    release(s)
    traffic = committed_traffic("step2")
    cells = prob["nx"] * prob["ny"]
    rate = cells * 64 / (ms / 1e3)
    return {"tblock": 2, "Mcell_updates_per_s": rate / 1e6, "ms_per_step": ms / 64,
            "vs_single_step": rate / single,
            "two_step_kernel": {"ms_per_launch": k_ms, "cells": k_cells, "steps_per_launch": 2,
                                "hbm_frac_of_528B_per_cell_update":
                                    ALG_BYTES["f64"] * k_cells * 2 / (k_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                                "traffic_bytes_per_cell_update": (None if traffic is None
                                                                  else traffic / k_cells / 2),
                                "traffic_gbs": None if traffic is None else traffic / (k_ms / 1e3) / 1e9}}


def vn_sweep(P):
    """The stability sweep of Sec. 4 on the GPU: spectral radius of the 33 x 33 amplification
    matrix in double-double for 64 states (the Fig. 2 state at lambda in [0.05, 3], T and u
    sweeps of Figs. 5, 6) x 64 phases in (0, pi]."""
    import numpy as np
    import torch
    V = (1.0, 1.92, 2.99, 4.49)
    cases = []
    for lam in np.linspace(0.05, 3.0, 32):
        cases.append(P.B.vn_case((2.0, 30.0, 0.0, 1.0), 3e-3, 1e-5, 1e-5, float(lam), 15, V))
    for T in np.linspace(1.0, 25.0, 16):
        cases.append(P.B.vn_case((2.0, 5.0, 0.0, float(T)), 3e-3, 1e-5, 1e-5, 0.0, 15, V))
    for u in np.linspace(0.0, 30.0, 16):
        cases.append(P.B.vn_case((2.0, float(u), 0.0, 1.0), 3e-3, 1e-5, 1e-5, 0.0, 15, V))
    phis = np.linspace(np.pi / 64, np.pi, 64)
    say(f"stability sweep: {len(cases)} x {len(phis)} matrices")
    P.B.fdlb_vn_sweep(cases[:2], phis[:2])  # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = P.B.fdlb_vn_sweep(cases, phis)
    sec = time.perf_counter() - t
    g = r.max(axis=1)
    return {"matrices": int(r.size), "seconds": sec, "matrices_per_s": r.size / sec,
            "arithmetic": "double-double", "converged": int(np.isfinite(r).sum()),
            "max_growth_fig2_lambda_0.05_and_3": [float(g[0]), float(g[31])],
            "max_growth_fig5_T_1_and_25": [float(g[32]), float(g[47])],
            "max_growth_fig6_u_0_and_30": [float(g[48]), float(g[63])]}


def host_cpu():
    model = platform.processor() or ""
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        m = re.search(r"Model name:\s*(.+)", txt)
        if m:
            model = m.group(1).strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=10).stdout.strip())
    except (OSError, subprocess.SubprocessError, ValueError):
        nproc = os.cpu_count()
    return model, nproc


def cpu_baseline(prob, fields, steps, rows):
    """The float64 oracle on the bottom `rows` rows of the headline grid (same sides:
    reflecting wall, inflow, outflow, top state), on one thread and on the host threads the
    job may use (at most 16, the machine's CPU share)."""
    import numpy as np

    import oracle
    model, nproc = host_cpu()
    nthr = max(1, min(16, nproc or 1))
    sub = dict(prob)
    sub["ny"] = min(rows, prob["ny"])
    flds = tuple(np.ascontiguousarray(f[:sub["ny"]]) for f in fields)
    oracle._lib()
    f0 = oracle.init_state(sub, flds)
    cells = sub["nx"] * sub["ny"]
    one_steps = max(1, steps // 8)
    t = time.perf_counter()
    oracle.run_f(sub, f0, one_steps, nthreads=1)
    dt1 = time.perf_counter() - t
    t = time.perf_counter()
    oracle.run_f(sub, f0, steps, nthreads=nthr)
    dt = time.perf_counter() - t
    # the stability analysis of Sec. 4 as the CPU tool does it (mpmath, 30 digits), one matrix
    import mpmath as mp

    from oracle import vonneumann as vn
    V = (1.0, 1.92, 2.99, 4.49)
    t = time.perf_counter()
    with mp.workdps(30):
        vel = vn.velocities(V)
        J = vn.dfeq_df(V, (2.0, 30.0, 0.0, 1.0), vel=vel)
        vn.spectral_radius(vn.amplification(V, (2.0, 30.0, 0.0, 1.0), 3e-3, 1e-5, 1e-5, mp.mpf(1.0), 0.5, 15,
                                            jac=J, vel=vel))
    vn_s = time.perf_counter() - t
    return {"value": cells * steps / dt / 1e6, "unit": "Mcell-updates/s", "cores": nthr, "kind": "oracle",
            "vn_mpmath_s_per_matrix": vn_s,
            "sample": f"{steps} steps of {sub['nx']}x{sub['ny']} (bottom rows of the headline grid, same sides) "
                      f"on {nthr} threads, {dt:.1f} s; {one_steps} steps on 1 thread, {dt1:.1f} s",
            "single_thread_value": cells * one_steps / dt1 / 1e6, "host_nproc": nproc, "host_cpu": model}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the slab decomposition over several "
              "GPUs is not built", file=sys.stderr)
        sys.exit(2)
    import torch

    import fdlb_inputs as fi
    import paper_0801_4169_amd as P
    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)

    prob, fields, _ = fi.cfg5_reflection(nx=args.nx, ny=args.ny)
    cells = prob["nx"] * prob["ny"]
    head = {}
    for pr in STORAGES:
        say(f"{pr}: {prob['nx']}x{prob['ny']}, {args.warmup} warmup + {args.steps} timed steps")
        r = headline_run(P, prob, fields, pr, args.steps, args.warmup, args.tile, graph_leg=(pr == "f64"))
        r["rate"] = cells * args.steps / (r["ms"] / 1e3)
        head[pr] = r
        say(f"{pr}: {r['ms'] / args.steps:.3f} ms/step, {r['rate'] / 1e9:.3f} Gcell-updates/s, "
            f"interior kernel {r['k_ms']:.3f} ms, non-physical={r['flag']}")

    r = head["f64"]
    achieved = ALG_BYTES["f64"] * r["k_cells"] / (r["k_ms"] / 1e3) / 1e9
    traffic = committed_traffic("f64")
    out = {
        "metric": "Mcell-updates/s FP32 vs FP64 at stated L1 error; % of HBM roofline",
        "value": r["rate"] / 1e6,
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": prob["name"], "nx": prob["nx"], "ny": prob["ny"], "dx": prob["dx"],
                   "dt": prob["dt"], "tau": prob["tau"], "lambda": prob["lam"], "inflow": list(fi.REFL_PRE),
                   "start": "incident shock smoothed over 2 cells", "storage": "f64", "tiling": r["tiling"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic / (r["k_ms"] / 1e3) / 1e9,
                     "kernel": "fdlb::step_kernel<double, interior tiles>",
                     "kernel_ms": r["k_ms"], "kernel_cells": r["k_cells"],
                     "alg_bytes_per_cell_update": ALG_BYTES["f64"],
                     # a plain copy of the same planes over the same tiles: the practical
                     # bandwidth of this access pattern, and the kernel's time against it
                     "copy_ceiling": {"ms": r["copy_ms"],
                                      "GBps": ALG_BYTES["f64"] * r["k_cells"] / (r["copy_ms"] / 1e3) / 1e9,
                                      "kernel_over_copy": r["copy_ms"] / r["k_ms"]}},
        "graph_replay_64": {"ms_per_step": r["graph64_ms"] / 64,
                            "Mcell_updates_per_s": cells * 64 / (r["graph64_ms"] / 1e3) / 1e6},
        "nonphysical": bool(r["flag"]),
    }
    for pr in ("f32", "f32dev"):
        o = head[pr]
        ent = {"value": o["rate"] / 1e6, "ms_per_step": o["ms"] / args.steps,
               "hbm_frac": ALG_BYTES[pr] * cells / (o["ms"] / args.steps / 1e3) / 1e9 / HBM_PEAK_GBS,
               "kernel_ms": o["k_ms"],
               "kernel_hbm_frac": ALG_BYTES[pr] * o["k_cells"] / (o["k_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS,
               "kernel_traffic_gbs": (None if committed_traffic(pr) is None
                                      else committed_traffic(pr) / (o["k_ms"] / 1e3) / 1e9),
               "copy_ceiling_ms": o["copy_ms"], "kernel_over_copy": o["copy_ms"] / o["k_ms"],
               "speedup_vs_f64": o["rate"] / head["f64"]["rate"], "nonphysical": bool(o["flag"]),
               "tiling": o["tiling"]}
        if physical(o["moments"]) and physical(head["f64"]["moments"]):
            ent["vs_f64_after_timed_steps"] = errors(o["moments"], head["f64"]["moments"])
        out[pr] = ent

    wanted = {int(c) for c in args.configs.split(",") if c.strip()}
    blocks = {}
    if 1 in wanted:
        blocks["cfg1"] = cfg1(P, fi)
    if 2 in wanted:
        blocks["cfg2"] = cfg2(P, fi)
    if 3 in wanted:
        blocks["cfg3"] = cfg3(P, fi)
    if 4 in wanted:
        blocks["cfg4"] = cfg4(P, fi)
    if 5 in wanted and args.nx == 8192 and args.ny == 2048:
        blocks["cfg5"] = cfg5_accuracy(P, fi, prob, fields, head, args.steps + args.warmup)
    if 5 in wanted:
        blocks.update(accuracy_blocks(P, fi, args.nx, args.ny))
    if not args.no_extras:
        out["two_step"] = two_step(P, prob, fields, head["f64"]["rate"])
        out["vn_sweep"] = vn_sweep(P)
    for pr in head:
        head[pr].pop("moments", None)
    if blocks:
        out["configs"] = blocks
    if args.copy_probe_mib > 0:
        a = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_mib"] = args.copy_probe_mib
        del a, b
    if args.cpu_steps > 0:
        say("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(prob, fields, args.cpu_steps, args.cpu_rows)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
