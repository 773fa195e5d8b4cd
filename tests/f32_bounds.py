"""Error bounds for the float32 storages, derived from their rounding rather than measured.

Each step stores every value s_q of a cell rounded to float32: the distribution f_q itself
(naive float32) or its deviation g_q = f_q - f^eq_q(M) from the equilibrium of the float64
moments M (deviation storage).  A stored value then carries an error |d_q| <= u |s_q|,
u = 2^-24, and the moments recovered from the cell (Eqs. n_eq, nu_eq, p_eq) move by, to
first order,

    dn = sum_q d_q
    du = sum_q d_q (v_q - u) / n
    dT = sum_q d_q (|v_q - u|^2 / 2 - T) / n        (T = E / n - |u|^2 / 2, E = sum f |v|^2 / 2)

so per step and cell |dn| <= u sum_q |s_q| and so on.  N steps that each add at most that
much, with nothing amplified, give N times the per-step bound; the per-cell bound is taken
as the larger of its values at the first and the last state.  The float64 arithmetic of a
step adds at most 64 ulp(1) of sum_q |f_q| per value, a term kept for completeness (it is
1e-10 of n at Mach 10, far below the float32 terms).

What the model leaves out, and so what a test against it assumes: amplification of errors
by the flow over the N steps (the runs checked are short), and, for naive float32, the
rounding of its float32 stencil arithmetic beyond the storage.  The states come from the
oracle alone.
"""
import numpy as np

import oracle

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def _per_step(prob, f, storages):
    """Per-cell first-order bounds of the (n, ux, uy, T) errors from one rounding of the
    state f (33, ny, nx), for each storage: {storage: {field: array}}, and the moments."""
    r, ux, uy, T = oracle.fields(prob, f)
    vx, vy = oracle.velocities(prob["v"])
    feq = oracle.init_state(prob, (r, ux, uy, T)) if "f32dev" in storages else None
    acc = {st: [np.zeros_like(r) for _ in range(4)] for st in storages}
    f_sum = np.zeros_like(r)
    for q in range(f.shape[0]):
        f_sum += np.abs(f[q])
        wx = np.abs(vx[q] - ux)
        wy = np.abs(vy[q] - uy)
        wT = np.abs(0.5 * ((vx[q] - ux) ** 2 + (vy[q] - uy) ** 2) - T)
        for st in storages:
            s = np.abs(f[q] - feq[q]) if st == "f32dev" else np.abs(f[q])
            a = acc[st]
            a[0] += s
            a[1] += s * wx
            a[2] += s * wy
            a[3] += s * wT
    a64 = 64.0 * U64 * f_sum
    vmax = float(np.max(np.hypot(vx, vy)))
    out = {}
    for st in storages:
        s_sum, fx, fy, fT = acc[st]
        out[st] = {"rho": U32 * s_sum + a64,
                   "ux": (U32 * fx + a64 * (vmax + np.abs(ux))) / r,
                   "uy": (U32 * fy + a64 * (vmax + np.abs(uy))) / r,
                   "T": (U32 * fT + a64 * (0.5 * (vmax + np.hypot(ux, uy)) ** 2 + T)) / r}
    return out, (r, ux, uy, T)


def bounds(prob, f_first, f_last, nsteps, storages=("f32", "f32dev")):
    """Bounds on the errors after nsteps, per storage, in the metrics of `rel_errors`: for
    rho and T (rel L1, rel Linf) = (sum|d| / sum|ref|, max|d| / max|ref|); for ux, uy
    (mean|d|, max|d|) over the largest velocity component of the reference (the last
    state's moments)."""
    a, _ = _per_step(prob, f_first, storages)
    b, ref = _per_step(prob, f_last, storages)
    r, ux, uy, T = ref
    uscale = max(float(np.max(np.abs(ux))), float(np.max(np.abs(uy))))
    out = {}
    for st in storages:
        per = {k: np.maximum(a[st][k], b[st][k]) * nsteps for k in a[st]}
        out[st] = {"rho": (float(per["rho"].sum() / np.abs(r).sum()), float(per["rho"].max() / np.abs(r).max())),
                   "ux": (float(per["ux"].mean() / uscale), float(per["ux"].max() / uscale)),
                   "uy": (float(per["uy"].mean() / uscale), float(per["uy"].max() / uscale)),
                   "T": (float(per["T"].sum() / np.abs(T).sum()), float(per["T"].max() / np.abs(T).max()))}
    return out


def rel_errors(m, ref):
    """(rel L1, rel Linf) of rho and T; of ux, uy the mean and max absolute error over the
    largest velocity component of the reference."""
    uscale = max(float(np.max(np.abs(ref[1]))), float(np.max(np.abs(ref[2]))))
    out = {}
    for name, a, b in zip(("rho", "ux", "uy", "T"), m, ref):
        d = np.abs(a - b)
        if name in ("ux", "uy"):
            out[name] = (float(np.mean(d)) / uscale, float(np.max(d)) / uscale)
        else:
            out[name] = (float(np.sum(d) / np.sum(np.abs(b))), float(np.max(d) / np.max(np.abs(b))))
    return out
