"""Benchmark of the FDLB hot path on one MI355X.

Workload (default): steady regular shock reflection on 8192 x 2048 cells, dx = dy = 2.5e-4,
dt = 1e-6, tau = 2e-6, 10000 steps: freestream (1, 10, 0, 0.5), a 30-degree incident shock
with the Rankine-Hugoniot post-shock state (gamma = 2) on the top side, reflecting wall at the
bottom, outflow on the right, artificial-viscosity amplitude lambda = 20.  (The paper's
Mach-20 inflow turns non-physical within a few steps with this scheme for every lambda, tau and
dt tried; freestream Mach 10 with lambda = 20 runs the full 10000 steps.)  A step is one
launch per tile kind that advances all 33 distributions of every cell by Eq. (dis_eq1).

Reported (one JSON line): cell-updates per second of the float64 path (`value`); the two
float32 storages ("f32": f in float32; "f32dev": moments in float64 and g = f - f^eq in
float32) with their speed-up and relative L1 difference to float64 after the same steps,
beside the difference a 1e-13 perturbation of the initial density makes in float64 (this
flow amplifies perturbations, so that is the floor any storage can reach); the 256-tube
ensemble in float64 and both float32 storages with per-instance L1 against float64; the
roofline of the dominant kernel (interior tiles, timed alone with HIP events) against the
MI355X HBM peak, HBM traffic from the committed counter summary when it matches the current
kernel source, and a plain copy of the same planes over the same tiles as the practical
ceiling of the access pattern; the storages' accuracy on the same grid with a Mach-5 inflow,
where float64 itself does not amplify rounding (`accuracy_mach5`); and the CPU oracle's
rate on a bounded slice of the same grid.
"""
import argparse
import hashlib
import json
import os
import re
import sys
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="all", choices=["all", "f64", "f32", "f32dev"])
    ap.add_argument("--nx", type=int, default=8192)
    ap.add_argument("--ny", type=int, default=2048)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--mach", type=float, default=10.0, help="freestream Mach number of the inflow")
    ap.add_argument("--lam", type=float, default=20.0, help="artificial-viscosity amplitude lambda")
    ap.add_argument("--ensemble-steps", type=int, default=5000, help="steps of the 256-tube ensemble (0: skip)")
    ap.add_argument("--accuracy-steps", type=int, default=2000,
                    help="steps of the storages' accuracy check on the Mach-5 flow (0: skip)")
    ap.add_argument("--no-sensitivity", action="store_true",
                    help="skip the perturbed float64 run that measures the flow's own sensitivity")
    ap.add_argument("--cpu-steps", type=int, default=100, help="oracle steps of the CPU baseline slice (0: skip)")
    ap.add_argument("--cpu-rows", type=int, default=256, help="rows of the CPU baseline slice")
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


def timed_run(P, prob, fields, precision, steps, warmup, tile):
    import torch
    s = P.Solver(prob, precision=precision, tile=tile)
    s.set_state(*fields)
    s.step(warmup)
    torch.cuda.synchronize()
    # the solver runs on torch's current stream, so these events bracket its launches
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    # the dominant kernel (interior tiles) alone, HIP events on the same stream
    k_ms = P.B.fdlb_time_kernel(s.ctx, 0, 50)
    k_cells = P.B.fdlb_tile_cells(s.ctx, 0)
    # the practical ceiling: a plain copy of the stored planes over the same tiles
    copy_ms = P.B.fdlb_copy_ceiling(s.ctx, 50)
    tiling = s.tiling
    m = s.moments(allow_nonphys=True)
    _, flag = s.diag()
    s.close()
    del s
    torch.cuda.empty_cache()
    return dict(ms=ms, moments=m, flag=flag, k_ms=k_ms, k_cells=k_cells, tiling=tiling, copy_ms=copy_ms)


def accuracy(P, fi, args):
    """The three storages on the same grid and sides with freestream Mach 5 and lambda = 2
    (a flow that does not amplify rounding: float64 with 1e-13 noise stays within 1e-11),
    relative L1 of (rho, ux, uy, T) against float64 after args.accuracy_steps steps."""
    import numpy as np
    prob, fields, _ = fi.reflection_8192x2048(lam=2.0, nx=args.nx, ny=args.ny, mach=5.0)
    n = args.accuracy_steps
    ref = timed_run(P, prob, fields, "f64", n, 0, args.tile)["moments"]
    rng = np.random.default_rng(1)
    pert = (fields[0] * (1.0 + 1e-13 * rng.standard_normal(fields[0].shape)),) + tuple(fields[1:])
    runs = {"f64_with_1e-13_noise": (pert, "f64"), "f32dev": (fields, "f32dev"), "f32": (fields, "f32")}
    out = {"workload": prob["name"], "lambda": 2.0, "steps": n}
    for name, (flds, pr) in runs.items():
        r = timed_run(P, prob, flds, pr, n, 0, args.tile)
        out[name] = {k: l1_rel(x, y) for k, x, y in zip(("rho", "ux", "uy", "T"), r["moments"], ref)}
        out[name]["nonphysical"] = bool(r["flag"])
    return out


def l1_rel(a, b):
    import numpy as np
    return float(np.sum(np.abs(a - b)) / max(np.sum(np.abs(b)), 1e-300))


def ensemble(P, steps):
    """The 256-tube ensemble in each storage: rate, and per-instance relative L1 of rho and T
    of both float32 storages against the float64 run (itself bit-identical to the oracle)."""
    import numpy as np
    import torch

    import fdlb_inputs as fi
    probs, _ = fi.ensemble_tubes()
    out = {"workload": "ensemble_256_tubes_seed0", "steps": steps}
    mom = {}
    for prec in ("f64", "f32", "f32dev"):
        b = P.BatchSolver([p for p, _ in probs], precision=prec)
        for i, (p, flds) in enumerate(probs):
            b.set_state(i, *flds)
        b.step(20)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.step(steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        mom[prec] = [b.moments(i, allow_nonphys=True) for i in range(len(probs))]
        physical = sum(int(np.all(np.isfinite(m[3])) and np.all(m[0] > 0) and np.all(m[3] > 0)) for m in mom[prec])
        cells = b.cells
        out[prec] = {"value": cells * steps / (ms / 1e3) / 1e6, "unit": "Mcell-updates/s", "ms_per_step": ms / steps,
                     "hbm_frac": ALG_BYTES[prec] * cells / (ms / steps / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "tiling": list(b.tiling), "instances_physical_at_end": physical}
        out["cells"] = cells
        b.close()
    for prec in ("f32", "f32dev"):
        l1 = np.array([[l1_rel(a[k], r[k]) for k in (0, 3)] for a, r in zip(mom[prec], mom["f64"])])
        out[prec]["l1_vs_f64_rho_T_median"] = [float(x) for x in np.median(l1, axis=0)]
        out[prec]["l1_vs_f64_rho_T_max"] = [float(x) for x in np.max(l1, axis=0)]
    return out


def cpu_baseline(prob, fields, steps, rows):
    """The float64 oracle on the bottom `rows` rows of the same grid (same sides: reflecting
    wall, inflow, outflow, top state), on the host threads the GPU job may use."""
    import numpy as np

    import oracle
    nthr = max(1, min(16, os.cpu_count() or 1))
    sub = dict(prob)
    sub["ny"] = min(rows, prob["ny"])
    flds = tuple(np.ascontiguousarray(f[:sub["ny"]]) for f in fields)
    oracle._lib()
    f0 = oracle.init_state(sub, flds)
    t = time.perf_counter()
    oracle.run_f(sub, f0, steps, nthreads=nthr)
    dt = time.perf_counter() - t
    cells = sub["nx"] * sub["ny"] * steps
    return {"value": cells / dt / 1e6, "unit": "Mcell-updates/s", "cores": nthr, "kind": "oracle",
            "sample": f"{steps} steps of {sub['nx']}x{sub['ny']} (bottom rows of the benchmark grid, same "
                      f"sides), {dt:.1f} s"}


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

    prob, fields, _ = fi.reflection_8192x2048(lam=args.lam, nx=args.nx, ny=args.ny, mach=args.mach)
    cells = prob["nx"] * prob["ny"]
    precs = ["f64", "f32", "f32dev"] if args.precision == "all" else [args.precision]
    res = {}
    for pr in precs:
        print(f"[bench] {pr}: {prob['nx']}x{prob['ny']}, {args.warmup} warmup + {args.steps} timed steps",
              file=sys.stderr, flush=True)
        r = timed_run(P, prob, fields, pr, args.steps, args.warmup, args.tile)
        r["rate"] = cells * args.steps / (r["ms"] / 1e3)
        res[pr] = r
        print(f"[bench] {pr}: {r['ms'] / args.steps:.3f} ms/step, {r['rate'] / 1e9:.3f} Gcell-updates/s, "
              f"interior kernel {r['k_ms']:.3f} ms, non-physical={r['flag']}", file=sys.stderr, flush=True)

    main_p = precs[0]
    r = res[main_p]
    ms_step = r["ms"] / args.steps
    achieved = ALG_BYTES[main_p] * r["k_cells"] / (r["k_ms"] / 1e3) / 1e9
    traffic = committed_traffic(main_p)
    out = {
        "metric": "Mcell-updates/s FP32 vs FP64 at stated L1 error; % of HBM roofline",
        "value": r["rate"] / 1e6,
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_p,
        "data": "synthetic",
        "config": {"workload": prob["name"], "nx": prob["nx"], "ny": prob["ny"], "dx": prob["dx"],
                   "dt": prob["dt"], "tau": prob["tau"], "lambda": prob["lam"], "storage": main_p,
                   "tiling": list(r["tiling"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic / (r["k_ms"] / 1e3) / 1e9,
                     "kernel": {"f64": "fdlb::step_kernel<double, interior tiles>",
                                "f32": "fdlb::step_kernel<float, interior tiles>",
                                "f32dev": "fdlb::step_kernel_dev<interior tiles>"}[main_p],
                     "kernel_ms": r["k_ms"], "kernel_cells": r["k_cells"],
                     "alg_bytes_per_cell_update": ALG_BYTES[main_p],
                     # a plain copy of the same planes over the same tiles: the practical
                     # bandwidth of this access pattern, and the kernel's time against it
                     "copy_ceiling": {"ms": r["copy_ms"],
                                      "GBps": ALG_BYTES[main_p] * r["k_cells"] / (r["copy_ms"] / 1e3) / 1e9,
                                      "kernel_over_copy": r["copy_ms"] / r["k_ms"]}},
        "nonphysical": bool(r["flag"]),
    }
    if "f64" in res and len(precs) > 1 and not args.no_sensitivity:
        import numpy as np
        print("[bench] f64 with 1e-13 noise in the initial density (sensitivity floor)", file=sys.stderr, flush=True)
        rng = np.random.default_rng(1)
        pert = (fields[0] * (1.0 + 1e-13 * rng.standard_normal(fields[0].shape)),) + tuple(fields[1:])
        rp_ = timed_run(P, prob, pert, "f64", args.steps, args.warmup, args.tile)
        out["f64_perturbed_l1_vs_f64_after_run"] = {k: l1_rel(x, y) for k, x, y in
                                                    zip(("rho", "ux", "uy", "T"), rp_["moments"], res["f64"]["moments"])}
    for pr in precs[1:]:
        o = res[pr]
        ent = {"value": o["rate"] / 1e6, "ms_per_step": o["ms"] / args.steps,
               "hbm_frac": ALG_BYTES[pr] * cells / (o["ms"] / args.steps / 1e3) / 1e9 / HBM_PEAK_GBS,
               "kernel_ms": o["k_ms"],
               "kernel_hbm_frac": ALG_BYTES[pr] * o["k_cells"] / (o["k_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS,
               "kernel_traffic_gbs": (None if committed_traffic(pr) is None
                                      else committed_traffic(pr) / (o["k_ms"] / 1e3) / 1e9),
               "copy_ceiling_ms": o["copy_ms"], "kernel_over_copy": o["copy_ms"] / o["k_ms"],
               "speedup_vs_f64": o["rate"] / res["f64"]["rate"], "nonphysical": bool(o["flag"]),
               "tiling": list(o["tiling"])}
        if "f64" in res:
            a, b = o["moments"], res["f64"]["moments"]
            ent["l1_vs_f64_after_run"] = {k: l1_rel(x, y) for k, x, y in zip(("rho", "ux", "uy", "T"), a, b)}
        out[pr] = ent
    if args.accuracy_steps > 0:
        print("[bench] accuracy on a flow that is not chaotic (Mach 5, lambda 2)", file=sys.stderr, flush=True)
        out["accuracy_mach5"] = accuracy(P, fi, args)
    if args.ensemble_steps > 0:
        print("[bench] ensemble", file=sys.stderr, flush=True)
        out["ensemble"] = ensemble(P, args.ensemble_steps)
    if args.copy_probe_mib > 0:
        a = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_mib"] = args.copy_probe_mib
        del a, b
    if args.cpu_steps > 0:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, fields, args.cpu_steps, args.cpu_rows)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
