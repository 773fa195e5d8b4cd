"""Benchmark of the FDLB hot path on one MI355X.

Workload: the Mach-20 steady regular reflection (inflow (1, 20, 0, 0.5), 30-degree incident
shock, reflecting wall at the bottom) on 8192 x 2048 cells, dx = dy = 2.5e-4, dt = 1e-6,
tau = 2e-6, lambda = 2, 10000 steps by default.  A step is one fused kernel launch that
advances all 33 distributions of every cell by Eq. (dis_eq1) of the paper.

Reported: cell-updates per second of the float64 path (the headline `value`) and of the
float32 path, the L1 difference between their final rho, u, T, the float64 step kernel's
achieved HBM bandwidth against the MI355X peak, and the CPU oracle's rate on a short slice
of the same workload.  Inputs are resident in HBM when the timed region starts; the timed
region is K steps between HIP events on the solver's stream.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
ALG_BYTES = {"f64": 2 * 33 * 8, "f32": 2 * 33 * 4}  # compulsory read + write of 33 planes per cell-update


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="both", choices=["both", "f64", "f32"])
    ap.add_argument("--nx", type=int, default=8192)
    ap.add_argument("--ny", type=int, default=2048)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle steps of the CPU baseline slice (0: skip)")
    ap.add_argument("--cpu-rows", type=int, default=512, help="rows of the CPU baseline slice")
    return ap.parse_args()


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
    m = s.moments(allow_nonphys=True)
    _, flag = s.diag()
    s.close()
    del s
    torch.cuda.empty_cache()
    return ms, m, flag


def l1_rel(a, b):
    import numpy as np
    return float(np.sum(np.abs(a - b)) / max(np.sum(np.abs(b)), 1e-300))


def cpu_baseline(prob, fields, steps, rows):
    """The float64 oracle on the first `rows` rows of the same grid (bottom wall, inflow,
    outflow and top state as in the full problem), all host threads."""
    import oracle
    import numpy as np
    nthr = os.cpu_count() or 1
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
            "sample": f"{steps} steps of {sub['nx']}x{sub['ny']} (bottom rows of the benchmark grid), "
                      f"{dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU decomposition is "
              "described in DESIGN.md and not built", file=sys.stderr)
        sys.exit(2)
    import torch
    import fdlb_inputs as fi
    import paper_0801_4169_amd as P
    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)

    prob, fields, _ = fi.reflection_8192x2048(nx=args.nx, ny=args.ny)
    cells = prob["nx"] * prob["ny"]
    precs = ["f64", "f32"] if args.precision == "both" else [args.precision]
    res = {}
    for pr in precs:
        print(f"[bench] {pr}: {prob['nx']}x{prob['ny']}, {args.warmup} warmup + {args.steps} timed steps",
              file=sys.stderr, flush=True)
        ms, m, flag = timed_run(P, prob, fields, pr, args.steps, args.warmup, args.tile)
        rate = cells * args.steps / (ms / 1e3)
        res[pr] = dict(ms=ms, moments=m, flag=flag, rate=rate)
        print(f"[bench] {pr}: {ms / args.steps:.3f} ms/step, {rate / 1e9:.3f} Gcell-updates/s, "
              f"non-physical={flag}", file=sys.stderr, flush=True)

    main_p = precs[0]
    r = res[main_p]
    ms_step = r["ms"] / args.steps
    achieved = ALG_BYTES[main_p] * cells / (ms_step / 1e3) / 1e9
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
                   "dt": prob["dt"], "tau": prob["tau"], "lambda": prob["lam"], "storage": main_p},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "fdlb::step_kernel", "alg_bytes_per_cell_update": ALG_BYTES[main_p]},
        "nonphysical": bool(r["flag"]),
    }
    for pr in precs[1:]:
        o = res[pr]
        ent = {"value": o["rate"] / 1e6, "ms_per_step": o["ms"] / args.steps,
               "hbm_frac": ALG_BYTES[pr] * cells / (o["ms"] / args.steps / 1e3) / 1e9 / HBM_PEAK_GBS,
               "speedup_vs_f64": o["rate"] / res["f64"]["rate"], "nonphysical": bool(o["flag"])}
        if "f64" in res:
            a, b = o["moments"], res["f64"]["moments"]
            ent["l1_vs_f64"] = {k: l1_rel(x, y) for k, x, y in zip(("rho", "ux", "uy", "T"), a, b)}
        out[pr] = ent
    if args.cpu_steps > 0:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prob, fields, args.cpu_steps, args.cpu_rows)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
