"""ctypes binding of libfdlb (include/fdlb.h): same names, argument marshalling only.

Every step of the hot path runs in the HIP library; this module converts Python and numpy
arguments to C types.  It raises ImportError at import time if the library is missing --
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FDLB_LIB selects another build of the same library (for example one built with
# different compile-time options); the default is the in-tree build.
LIB_PATH = os.environ.get("FDLB_LIB") or os.path.join(HERE, "libfdlb.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libfdlb.so not built ({LIB_PATH}); run __graft_entry__.build() or "
                      "python paper_0801_4169_amd/build.py")

# torch carries its own HIP and HSA runtimes.  Loading libfdlb first would bring in the
# system ones as well, and two HSA runtimes in one process do not share devices or memory
# (allocations then fail).  With torch loaded first, libfdlb's libamdhip64 dependency
# resolves by soname to torch's copy, and both use the same runtime.
import torch  # noqa: E402,F401  (imported for its HIP runtime, before the library)

_lib = ctypes.CDLL(LIB_PATH)

FDLB_OK, FDLB_EINVAL, FDLB_ENOMEM, FDLB_EDEVICE, FDLB_ENONPHYS, FDLB_ESTATE = range(6)
FDLB_F64, FDLB_F32, FDLB_F32_DEV = 0, 1, 2
FDLB_BC_PERIODIC, FDLB_BC_OUTFLOW, FDLB_BC_DIRICHLET, FDLB_BC_WALL = range(4)
PRECISIONS = {"f64": FDLB_F64, "f32": FDLB_F32, "f32dev": FDLB_F32_DEV}


class fdlb_bc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad_", ctypes.c_int32), ("rho", ctypes.c_double),
                ("ux", ctypes.c_double), ("uy", ctypes.c_double), ("T", ctypes.c_double),
                ("lo_kind", ctypes.c_int32), ("pad2_", ctypes.c_int32), ("lo_rho", ctypes.c_double),
                ("lo_ux", ctypes.c_double), ("lo_uy", ctypes.c_double), ("lo_T", ctypes.c_double),
                ("split", ctypes.c_double), ("split_rate", ctypes.c_double)]


class fdlb_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("dt", ctypes.c_double), ("tau", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("v", ctypes.c_double * 4), ("bc", fdlb_bc * 4), ("precision", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("lines", ctypes.c_int32), ("tblock", ctypes.c_int32),
                ("theta_fixed", ctypes.c_int32), ("pad_", ctypes.c_int32), ("theta_value", ctypes.c_double)]


class fdlb_vn_case(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("ux", ctypes.c_double), ("uy", ctypes.c_double), ("T", ctypes.c_double),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double), ("tau", ctypes.c_double),
                ("theta", ctypes.c_double), ("v", ctypes.c_double * 4), ("lines", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class FdlbError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{fdlb_strerror(status)} (status {status}){': ' + msg if msg else ''}")


_P = ctypes.POINTER(fdlb_params)
_CTX = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)

_sigs = {
    "fdlb_required_bytes": (ctypes.c_size_t, [_P]),
    "fdlb_batch_required_bytes": (ctypes.c_size_t, [ctypes.c_int32, _P]),
    "fdlb_create": (ctypes.c_int, [_P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(_CTX)]),
    "fdlb_batch_create": (ctypes.c_int, [ctypes.c_int32, _P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.POINTER(_CTX)]),
    "fdlb_set_state": (ctypes.c_int, [_CTX, _DP, _DP, _DP, _DP]),
    "fdlb_set_state_device": (ctypes.c_int, [_CTX, ctypes.c_void_p]),
    "fdlb_batch_set_state": (ctypes.c_int, [_CTX, ctypes.c_int32, _DP, _DP, _DP, _DP]),
    "fdlb_step": (ctypes.c_int, [_CTX, ctypes.c_int64]),
    "fdlb_batch_step": (ctypes.c_int, [_CTX, ctypes.c_int64]),
    "fdlb_get_moments": (ctypes.c_int, [_CTX, _DP, _DP, _DP, _DP]),
    "fdlb_batch_get_moments": (ctypes.c_int, [_CTX, ctypes.c_int32, _DP, _DP, _DP, _DP]),
    "fdlb_get_moments_device": (ctypes.c_int, [_CTX, ctypes.c_void_p]),
    "fdlb_f_bytes": (ctypes.c_size_t, [_CTX]),
    "fdlb_get_f": (ctypes.c_int, [_CTX, ctypes.c_void_p, ctypes.c_size_t]),
    "fdlb_set_f": (ctypes.c_int, [_CTX, ctypes.c_void_p, ctypes.c_size_t]),
    "fdlb_diag": (ctypes.c_int, [_CTX, _DP, ctypes.POINTER(ctypes.c_int32)]),
    "fdlb_diag_noalloc": (ctypes.c_int, [_CTX, _DP, ctypes.POINTER(ctypes.c_int32)]),
    "fdlb_steps_done": (ctypes.c_int64, [_CTX]),
    "fdlb_set_clock": (ctypes.c_int, [_CTX, ctypes.c_int64]),
    "fdlb_destroy": (None, [_CTX]),
    "fdlb_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "fdlb_last_error": (ctypes.c_char_p, [_CTX]),
    "fdlb_tile_shapes": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
    "fdlb_set_tiling": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.c_int32]),
    "fdlb_get_tiling": (ctypes.c_int, [_CTX, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "fdlb_tile_cells": (ctypes.c_int64, [_CTX, ctypes.c_int32]),
    "fdlb_time_kernel": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]),
    "fdlb_copy_ceiling": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]),
    "fdlb_vn_sweep": (ctypes.c_int, [ctypes.POINTER(fdlb_vn_case), ctypes.c_int32, _DP, ctypes.c_int32, _DP,
                                     ctypes.c_void_p]),
    "fdlb_vn_matrix": (ctypes.c_int, [ctypes.POINTER(fdlb_vn_case), ctypes.c_double, _DP, ctypes.c_void_p]),
    "fdlb_autotune": (ctypes.c_int, [_CTX, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]),
}
for _name, (_res, _args) in _sigs.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_sigs)


def fdlb_strerror(status):
    return _lib.fdlb_strerror(int(status)).decode()


def _check(status, ctx=None):
    if status != FDLB_OK:
        msg = _lib.fdlb_last_error(ctx).decode()
        raise FdlbError(status, msg)


def _f64(a, n=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _ptr(a):
    return a.ctypes.data_as(_DP)


def make_params(prob, precision="f64", tile=0, tblock=1, theta=None):
    """fdlb_params from a problem dict: nx, ny, dx, dy, dt, tau, lam, v, bc (4 kinds),
    bc_state (4 x (rho, ux, uy, T)), lower (4 x None or (kind, state, split, split_rate)),
    lines (bits of the terms of Eq. (dis_eq1) kept; default the full scheme).  ``tblock``:
    steps per pass over memory (1, or 2 for float64: interior tiles take two steps per
    launch).  ``theta``: None for the switching function of Eq. (add4), or the value theta
    of line IV is frozen at (Sec. 4)."""
    p = fdlb_params()
    p.nx, p.ny = int(prob["nx"]), int(prob["ny"])
    p.dx, p.dy = float(prob["dx"]), float(prob.get("dy", prob["dx"]))
    p.dt, p.tau, p.lambda_ = float(prob["dt"]), float(prob["tau"]), float(prob["lam"])
    for k in range(4):
        p.v[k] = float(prob["v"][k])
        p.bc[k].kind = int(prob["bc"][k])
        st = prob.get("bc_state", [(1.0, 0.0, 0.0, 1.0)] * 4)[k]
        p.bc[k].rho, p.bc[k].ux, p.bc[k].uy, p.bc[k].T = map(float, st)
        lo = prob.get("lower", (None,) * 4)[k]
        if lo is not None:
            kind, lst, split, rate = lo
            p.bc[k].lo_kind = int(kind)
            p.bc[k].lo_rho, p.bc[k].lo_ux, p.bc[k].lo_uy, p.bc[k].lo_T = map(float, lst)
            p.bc[k].split, p.bc[k].split_rate = float(split), float(rate)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.tile = int(tile)
    p.lines = int(prob.get("lines", 15))
    p.tblock = int(tblock)
    p.theta_fixed = 0 if theta is None else 1
    p.theta_value = 0.0 if theta is None else float(theta)
    return p


def fdlb_required_bytes(params):
    return int(_lib.fdlb_required_bytes(ctypes.byref(params)))


def fdlb_batch_required_bytes(params_list):
    arr = (fdlb_params * len(params_list))(*params_list)
    return int(_lib.fdlb_batch_required_bytes(len(params_list), arr))


def fdlb_create(params, stream, arena_ptr, arena_bytes):
    ctx = _CTX()
    _check(_lib.fdlb_create(ctypes.byref(params), ctypes.c_void_p(stream), ctypes.c_void_p(arena_ptr),
                            int(arena_bytes), ctypes.byref(ctx)))
    return ctx


def fdlb_batch_create(params_list, stream, arena_ptr, arena_bytes):
    arr = (fdlb_params * len(params_list))(*params_list)
    ctx = _CTX()
    _check(_lib.fdlb_batch_create(len(params_list), arr, ctypes.c_void_p(stream), ctypes.c_void_p(arena_ptr),
                                  int(arena_bytes), ctypes.byref(ctx)))
    return ctx


def fdlb_set_state(ctx, rho, ux, uy, T, n):
    a = [_f64(x, n) for x in (rho, ux, uy, T)]
    _check(_lib.fdlb_set_state(ctx, *[_ptr(x) for x in a]), ctx)


def fdlb_set_state_device(ctx, fields_ptr):
    _check(_lib.fdlb_set_state_device(ctx, ctypes.c_void_p(fields_ptr)), ctx)


def fdlb_batch_set_state(ctx, i, rho, ux, uy, T, n):
    a = [_f64(x, n) for x in (rho, ux, uy, T)]
    _check(_lib.fdlb_batch_set_state(ctx, int(i), *[_ptr(x) for x in a]), ctx)


def fdlb_step(ctx, nsteps):
    _check(_lib.fdlb_step(ctx, int(nsteps)), ctx)


def fdlb_batch_step(ctx, nsteps):
    _check(_lib.fdlb_batch_step(ctx, int(nsteps)), ctx)


def _get4(fn, ctx, n, *lead):
    outs = [np.empty(n, dtype=np.float64) for _ in range(4)]
    st = fn(ctx, *lead, *[_ptr(o) for o in outs])
    return st, outs


def fdlb_get_moments(ctx, n, allow_nonphys=False):
    st, outs = _get4(_lib.fdlb_get_moments, ctx, n)
    if not (allow_nonphys and st == FDLB_ENONPHYS):
        _check(st, ctx)
    return outs, st == FDLB_ENONPHYS


def fdlb_batch_get_moments(ctx, i, n, allow_nonphys=False):
    st, outs = _get4(_lib.fdlb_batch_get_moments, ctx, n, int(i))
    if not (allow_nonphys and st == FDLB_ENONPHYS):
        _check(st, ctx)
    return outs, st == FDLB_ENONPHYS


def fdlb_get_moments_device(ctx, fields_ptr):
    _check(_lib.fdlb_get_moments_device(ctx, ctypes.c_void_p(fields_ptr)), ctx)


def fdlb_f_bytes(ctx):
    return int(_lib.fdlb_f_bytes(ctx))


def fdlb_get_f(ctx, out, allow_nonphys=False):
    """Fills the numpy array `out` (33 * ny * nx of the storage dtype)."""
    st = _lib.fdlb_get_f(ctx, out.ctypes.data_as(ctypes.c_void_p), out.nbytes)
    if not (allow_nonphys and st == FDLB_ENONPHYS):
        _check(st, ctx)
    return st == FDLB_ENONPHYS


def fdlb_set_f(ctx, f):
    f = np.ascontiguousarray(f)
    _check(_lib.fdlb_set_f(ctx, f.ctypes.data_as(ctypes.c_void_p), f.nbytes), ctx)


def fdlb_diag(ctx):
    sums = np.zeros(4)
    flag = ctypes.c_int32(0)
    _check(_lib.fdlb_diag(ctx, _ptr(sums), ctypes.byref(flag)), ctx)
    return sums, bool(flag.value)


def fdlb_diag_noalloc(ctx):
    """fdlb_diag through the library's fixed scratch (the call allocates no device memory)."""
    sums = np.zeros(4)
    flag = ctypes.c_int32(0)
    _check(_lib.fdlb_diag_noalloc(ctx, _ptr(sums), ctypes.byref(flag)), ctx)
    return sums, bool(flag.value)


def fdlb_steps_done(ctx):
    return int(_lib.fdlb_steps_done(ctx))


def fdlb_set_clock(ctx, steps):
    _check(_lib.fdlb_set_clock(ctx, int(steps)), ctx)


def fdlb_destroy(ctx):
    _lib.fdlb_destroy(ctx)


def fdlb_set_tiling(ctx, shape_id, group):
    _check(_lib.fdlb_set_tiling(ctx, int(shape_id), int(group)), ctx)


def fdlb_get_tiling(ctx):
    sh, g = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(_lib.fdlb_get_tiling(ctx, ctypes.byref(sh), ctypes.byref(g)), ctx)
    return sh.value, g.value


def fdlb_autotune(ctx, trial_steps, shape_ids=(), groups=()):
    """Returns (shape_id, group, best ms per step) after tuning in place."""
    sh = (ctypes.c_int32 * max(1, len(shape_ids)))(*shape_ids)
    gr = (ctypes.c_int32 * max(1, len(groups)))(*groups)
    best = ctypes.c_float(0)
    _check(_lib.fdlb_autotune(ctx, int(trial_steps), sh, len(shape_ids), gr, len(groups), ctypes.byref(best)), ctx)
    s, g = fdlb_get_tiling(ctx)
    return s, g, best.value


def fdlb_tile_cells(ctx, kind):
    return int(_lib.fdlb_tile_cells(ctx, int(kind)))


def fdlb_time_kernel(ctx, kind, launches):
    """Milliseconds per launch of one tile kind (-1: whole step); the state is unchanged."""
    ms = ctypes.c_float(0)
    _check(_lib.fdlb_time_kernel(ctx, int(kind), int(launches), ctypes.byref(ms)), ctx)
    return ms.value


def fdlb_copy_ceiling(ctx, launches):
    ms = ctypes.c_float(0.0)
    _check(_lib.fdlb_copy_ceiling(ctx, int(launches), ctypes.byref(ms)), ctx)
    return float(ms.value)


def fdlb_tile_shapes():
    buf = (ctypes.c_int32 * 64)()
    n = _lib.fdlb_tile_shapes(buf, 32)
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(n)]


def vn_case(state, dx, dt, tau, theta=0.0, lines=15, v=(1.0, 1.92, 2.99, 4.49)):
    """fdlb_vn_case of a uniform state (rho, ux, uy, T) and the scheme's parameters."""
    c = fdlb_vn_case()
    c.rho, c.ux, c.uy, c.T = map(float, state)
    c.dx, c.dt, c.tau, c.theta = float(dx), float(dt), float(tau), float(theta)
    for k in range(4):
        c.v[k] = float(v[k])
    c.lines = int(lines)
    return c


def fdlb_vn_sweep(cases, phis, stream=None):
    """Spectral radii of G(phi) (Eq. gi_j_eq) as an array (ncases, nphi)."""
    arr = (fdlb_vn_case * len(cases))(*cases)
    ph = np.ascontiguousarray(np.asarray(phis, dtype=np.float64))
    out = np.zeros((len(cases), len(ph)))
    _check(_lib.fdlb_vn_sweep(arr, len(cases), _ptr(ph), len(ph), _ptr(out), ctypes.c_void_p(stream)))
    return out


def fdlb_vn_matrix(case, phi, stream=None):
    """G(phi) as (33, 33, 4) float64: real hi, real lo, imaginary hi, imaginary lo."""
    out = np.zeros((33, 33, 4))
    _check(_lib.fdlb_vn_matrix(ctypes.byref(case), float(phi), _ptr(out), ctypes.c_void_p(stream)))
    return out
