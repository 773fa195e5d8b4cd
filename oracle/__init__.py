"""CPU oracle of the FDLB scheme (arXiv:0801.4169) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library neither links nor calls it, and
the two share no code: the only common Python dependency is ``fdlb_inputs``, which makes
parameters and initial fields and holds none of the method's arithmetic.

``fdlb_oracle.c`` holds the scheme itself (plain loops, float64, no fused multiply-add);
this module compiles it with gcc and exposes it through ctypes.  A second build of the
same source in __float128 (``quad=True``) measures the oracle's own rounding.

Companion modules: ``oracle.riemann`` (exact Riemann solver, any gamma) and
``oracle.vonneumann`` (amplification matrix of Eq. (gi_j_eq), extended precision).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fdlb_oracle.c")
LIBS = {False: os.path.join(HERE, "liboracle_f64.so"), True: os.path.join(HERE, "liboracle_f128.so")}
NQ = 33


def build(verbose=False):
    """Compile both oracle builds (float64 and __float128) in place."""
    base = ["gcc", "-O3", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
            "-fopenmp", "-Wall", "-Wno-unknown-pragmas"]
    for quad, lib in LIBS.items():
        cmd = base + (["-DORC_QUAD"] if quad else []) + [SRC, "-o", lib + ".tmp", "-lm"]
        if quad:
            cmd.append("-lquadmath")
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("oracle build failed:\n" + " ".join(cmd) + "\n" + r.stderr)
        if verbose and r.stderr:
            print(r.stderr)
        os.replace(lib + ".tmp", lib)


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dt", ctypes.c_double),
        ("tau", ctypes.c_double), ("lam", ctypes.c_double),
        ("v", ctypes.c_double * 4),
        ("bc", ctypes.c_int32 * 4),
        ("bc_state", (ctypes.c_double * 4) * 4),
        ("lines", ctypes.c_int32),
        ("theta_fixed", ctypes.c_int32),
        ("theta_value", ctypes.c_double),
        ("bc_lo", ctypes.c_int32 * 4),
        ("bc_lo_state", (ctypes.c_double * 4) * 4),
        ("split", ctypes.c_double * 4),
        ("split_rate", ctypes.c_double * 4),
        ("step0", ctypes.c_int64),
    ]


_libs = {}


def _lib(quad=False):
    if quad not in _libs:
        path = LIBS[quad]
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(Params)
        lib.orc_velocities.argtypes = [dp, dp, dp]
        lib.orc_weights.argtypes = [dp, ctypes.c_double, dp]
        lib.orc_feq.argtypes = [dp] + [ctypes.c_double] * 4 + [dp]
        lib.orc_moments.argtypes = [dp, dp, dp]
        lib.orc_mirror.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.orc_mirror.restype = ctypes.c_int
        lib.orc_init_state.argtypes = [pp, dp, dp, dp, dp, dp]
        lib.orc_run_f.argtypes = [pp, dp, ctypes.c_long, ctypes.c_int, ctypes.POINTER(ctypes.c_long)]
        lib.orc_run_state.argtypes = [pp, dp, dp, dp, dp, ctypes.c_long, ctypes.c_int, dp, dp, dp, dp,
                                      ctypes.POINTER(ctypes.c_long)]
        lib.orc_fields.argtypes = [pp, dp, dp, dp, dp, dp]
        lib.orc_real_bytes.restype = ctypes.c_int
        _libs[quad] = lib
    return _libs[quad]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64))


def params(prob, lines=None, theta_fixed=False, theta_value=0.0, step0=0):
    """ctypes parameter block from a problem dict (see ``fdlb_inputs.problem``); ``step0``
    is the step number of the first step (time-dependent side segments); ``lines`` the
    terms of Eq. (dis_eq1) kept (bits for lines I..IV), by default the problem's own
    (``prob["lines"]``, else the full scheme)."""
    p = Params()
    p.nx, p.ny = prob["nx"], prob["ny"]
    p.dx, p.dy, p.dt, p.tau, p.lam = prob["dx"], prob["dy"], prob["dt"], prob["tau"], prob["lam"]
    for k in range(4):
        p.v[k] = prob["v"][k]
        p.bc[k] = prob["bc"][k]
        for c in range(4):
            p.bc_state[k][c] = prob["bc_state"][k][c]
    p.lines = int(prob.get("lines", 15)) if lines is None else lines
    p.theta_fixed = 1 if theta_fixed else 0
    p.theta_value = theta_value
    for k, seg in enumerate(prob.get("lower", (None,) * 4)):
        if seg is None:
            continue
        kind, state, split, rate = seg
        p.bc_lo[k] = kind
        for c in range(4):
            p.bc_lo_state[k][c] = state[c]
        p.split[k], p.split_rate[k] = split, rate
    p.step0 = step0
    return p


def velocities(v):
    v = _vec(v)
    vx = np.zeros(NQ)
    vy = np.zeros(NQ)
    _lib().orc_velocities(_dp(v), _dp(vx), _dp(vy))
    return vx, vy


def mirror(axis, q):
    return _lib().orc_mirror(axis, q)


def weights(v, T):
    """(F_0, F_1..F_4) of Eqs. (fk_eq1), (f0_eq) at theta = T."""
    v = _vec(v)
    F = np.zeros(5)
    _lib().orc_weights(_dp(v), float(T), _dp(F))
    return F


def feq(v, n, ux, uy, T):
    v = _vec(v)
    out = np.zeros(NQ)
    _lib().orc_feq(_dp(v), float(n), float(ux), float(uy), float(T), _dp(out))
    return out


def moments(v, f):
    """(n, ux, uy, T, P) of one 33-vector."""
    v = _vec(v)
    f = _vec(f)
    out = np.zeros(5)
    _lib().orc_moments(_dp(v), _dp(f), _dp(out))
    return out


def _fields_in(prob, fields):
    ny, nx = prob["ny"], prob["nx"]
    return [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (ny, nx))) for a in fields]


def init_state(prob, fields):
    """f := f^eq of the fields, shape (33, ny, nx)."""
    p = params(prob)
    r, u, w, T = _fields_in(prob, fields)
    f = np.zeros((NQ, prob["ny"], prob["nx"]))
    if _lib().orc_init_state(ctypes.byref(p), _dp(r), _dp(u), _dp(w), _dp(T), _dp(f)) != 0:
        raise ValueError("invalid problem")
    return f


def run_f(prob, f, nsteps, nthreads=1, **kw):
    """Advances f (33, ny, nx) by nsteps; returns (f_new, first_bad_step or -1)."""
    p = params(prob, **kw)
    f = np.ascontiguousarray(np.array(f, dtype=np.float64, copy=True))
    fb = ctypes.c_long(-1)
    if _lib().orc_run_f(ctypes.byref(p), _dp(f), int(nsteps), int(nthreads), ctypes.byref(fb)) != 0:
        raise ValueError("invalid problem")
    return f, fb.value


def run_state(prob, fields, nsteps, nthreads=1, quad=False, **kw):
    """Equilibrium start from the fields, nsteps, then (rho, ux, uy, T) and the first
    non-physical step (-1 if none)."""
    p = params(prob, **kw)
    r, u, w, T = _fields_in(prob, fields)
    outs = [np.zeros((prob["ny"], prob["nx"])) for _ in range(4)]
    fb = ctypes.c_long(-1)
    rc = _lib(quad).orc_run_state(ctypes.byref(p), _dp(r), _dp(u), _dp(w), _dp(T), int(nsteps),
                                  int(nthreads), *[_dp(o) for o in outs], ctypes.byref(fb))
    if rc != 0:
        raise ValueError("invalid problem")
    return tuple(outs), fb.value


def fields(prob, f):
    """(rho, ux, uy, T) of f (33, ny, nx)."""
    p = params(prob)
    f = np.ascontiguousarray(np.asarray(f, dtype=np.float64))
    outs = [np.zeros((prob["ny"], prob["nx"])) for _ in range(4)]
    _lib().orc_fields(ctypes.byref(p), _dp(f), *[_dp(o) for o in outs])
    return tuple(outs)
