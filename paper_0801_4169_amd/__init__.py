"""MI355X-native finite-difference lattice Boltzmann (FDLB) solver for compressible flow at
high Mach number -- the model of Gan, Xu, Zhang, Yu and Li (arXiv:0801.4169).

The hot path (one fused HIP kernel per time step) lives in ``libfdlb.so``; see
``include/fdlb.h`` for the C interface.  This package holds the ctypes binding (same names
as the C interface) and two small convenience classes that use PyTorch only for device
memory and the stream.
"""
from __future__ import annotations

import numpy as np

from . import _binding as B
from ._binding import (FDLB_BC_DIRICHLET, FDLB_BC_OUTFLOW, FDLB_BC_PERIODIC, FDLB_BC_WALL, FDLB_F32, FDLB_F32_DEV,
                       FDLB_F64, FDLB_EINVAL, FDLB_ENONPHYS, FDLB_ESTATE, FdlbError, fdlb_tile_shapes, make_params)

__all__ = ["Solver", "BatchSolver", "FdlbError", "make_params", "fdlb_tile_shapes", "B"]

NQ = 33


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the FDLB solver needs a HIP device")
    return torch


class Solver:
    """One problem on one GPU.  ``prob`` is a problem dict (nx, ny, dx, dy, dt, tau, lam, v,
    bc, bc_state); ``precision`` is "f64", "f32" or "f32dev" (deviation storage);
    ``tile`` a shape id (0 = default); ``tblock`` steps per pass over memory (2: float64
    interior tiles take two steps per launch, the same values as single steps); ``theta``
    None, or the value theta of line IV is frozen at (Sec. 4 linearises the scheme so)."""

    def __init__(self, prob, precision="f64", tile=0, device="cuda:0", tblock=1, theta=None):
        torch = _torch()
        self.prob = dict(prob)
        self.params = make_params(prob, precision, tile, tblock, theta)
        self.nx, self.ny = self.params.nx, self.params.ny
        self.ncell = self.nx * self.ny
        self.dtype = np.float64 if self.params.precision == FDLB_F64 else np.float32
        self.dev = self.params.precision == FDLB_F32_DEV
        nbytes = B.fdlb_required_bytes(self.params)
        if nbytes == 0:
            raise FdlbError(FDLB_EINVAL, "invalid parameters")
        self.device = torch.device(device)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = B.fdlb_create(self.params, self.stream.cuda_stream, self.arena.data_ptr(), nbytes)

    # -- state ------------------------------------------------------------------------
    def set_state(self, rho, ux, uy, T):
        B.fdlb_set_state(self.ctx, rho, ux, uy, T, self.ncell)

    def set_state_device(self, fields):
        """fields: float64 CUDA tensor of shape (4, ny, nx) (rho, ux, uy, T)."""
        torch = _torch()
        assert fields.dtype == torch.float64 and fields.is_contiguous() and fields.numel() == 4 * self.ncell
        B.fdlb_set_state_device(self.ctx, fields.data_ptr())
        self._keep = fields

    def step(self, n=1):
        B.fdlb_step(self.ctx, n)

    def moments(self, allow_nonphys=False):
        """(rho, ux, uy, T) as numpy arrays of shape (ny, nx); raises FdlbError on a
        non-physical state unless allow_nonphys."""
        outs, _ = B.fdlb_get_moments(self.ctx, self.ncell, allow_nonphys)
        return tuple(o.reshape(self.ny, self.nx) for o in outs)

    def moments_device(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((4, self.ny, self.nx), dtype=torch.float64, device=self.device)
        B.fdlb_get_moments_device(self.ctx, out.data_ptr())
        return out

    def get_f(self, allow_nonphys=False):
        """The stored state: f (33, ny, nx); for deviation storage the pair (g float32
        (33, ny, nx), moments float64 (4, ny, nx))."""
        if self.dev:
            buf = np.empty(B.fdlb_f_bytes(self.ctx), dtype=np.uint8)
            B.fdlb_get_f(self.ctx, buf, allow_nonphys)
            k = NQ * self.ncell * 4
            g = buf[:k].view(np.float32).reshape(NQ, self.ny, self.nx).copy()
            m = buf[k:].copy().view(np.float64).reshape(4, self.ny, self.nx)
            return g, m
        out = np.empty((NQ, self.ny, self.nx), dtype=self.dtype)
        B.fdlb_get_f(self.ctx, out, allow_nonphys)
        return out

    def set_f(self, f):
        if self.dev:
            g, m = f
            g = np.ascontiguousarray(np.asarray(g, dtype=np.float32))
            m = np.ascontiguousarray(np.asarray(m, dtype=np.float64))
            assert g.shape == (NQ, self.ny, self.nx) and m.shape == (4, self.ny, self.nx)
            B.fdlb_set_f(self.ctx, np.concatenate([g.view(np.uint8).ravel(), m.view(np.uint8).ravel()]))
            return
        f = np.ascontiguousarray(np.asarray(f, dtype=self.dtype))
        assert f.shape == (NQ, self.ny, self.nx)
        B.fdlb_set_f(self.ctx, f)

    def diag(self):
        return B.fdlb_diag(self.ctx)

    @property
    def tiling(self):
        """(tile shape id, dispatch-group width) of the step launch."""
        return B.fdlb_get_tiling(self.ctx)

    def set_tiling(self, shape_id, group):
        B.fdlb_set_tiling(self.ctx, shape_id, group)

    def autotune(self, trial_steps=20, shape_ids=(), groups=(), cache=None):
        """Times the tiling candidates on the current state (which it leaves unchanged) and
        keeps the fastest.  With ``cache`` (a JSON file path) a result for the same grid,
        precision and device is reused instead of re-timed."""
        return _autotune(self, trial_steps, shape_ids, groups, cache,
                         key=f"{self.params.precision}:{self.nx}x{self.ny}")

    @property
    def steps_done(self):
        return B.fdlb_steps_done(self.ctx)

    def set_clock(self, steps):
        """Step count that times moving side segments (e.g. after restoring a checkpoint)."""
        B.fdlb_set_clock(self.ctx, steps)

    def close(self):
        if getattr(self, "ctx", None):
            B.fdlb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autotune(solver, trial_steps, shape_ids, groups, cache, key):
    import json
    import os
    torch = _torch()
    key = f"{torch.cuda.get_device_name(solver.device)}:{key}"
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
    if key in table:
        sh, g = table[key]["shape"], table[key]["group"]
        B.fdlb_set_tiling(solver.ctx, sh, g)
        return sh, g, table[key]["ms"]
    sh, g, ms = B.fdlb_autotune(solver.ctx, trial_steps, shape_ids, groups)
    if cache:
        table[key] = {"shape": sh, "group": g, "ms": ms}
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return sh, g, ms


class BatchSolver:
    """k independent problems advanced by one launch per step (per tile kind).  ``tblock``
    as for Solver, for every instance (float64); ``thetas`` None, or per instance None or
    the value theta of line IV is frozen at (Sec. 4)."""

    def __init__(self, probs, precision="f32", tile=0, device="cuda:0", tblock=1, thetas=None):
        torch = _torch()
        thetas = thetas if thetas is not None else [None] * len(probs)
        self.params = [make_params(p, precision, tile, tblock, th) for p, th in zip(probs, thetas)]
        self.sizes = [(p.ny, p.nx) for p in self.params]
        self.dtype = np.float64 if self.params[0].precision == FDLB_F64 else np.float32
        nbytes = B.fdlb_batch_required_bytes(self.params)
        if nbytes == 0:
            raise FdlbError(FDLB_EINVAL, "invalid parameters")
        self.device = torch.device(device)
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = B.fdlb_batch_create(self.params, self.stream.cuda_stream, self.arena.data_ptr(), nbytes)

    @property
    def cells(self):
        return sum(ny * nx for ny, nx in self.sizes)

    def set_state(self, i, rho, ux, uy, T):
        ny, nx = self.sizes[i]
        B.fdlb_batch_set_state(self.ctx, i, rho, ux, uy, T, ny * nx)

    def step(self, n=1):
        B.fdlb_batch_step(self.ctx, n)

    def moments(self, i, allow_nonphys=False):
        ny, nx = self.sizes[i]
        outs, _ = B.fdlb_batch_get_moments(self.ctx, i, ny * nx, allow_nonphys)
        return tuple(o.reshape(ny, nx) for o in outs)

    def diag(self):
        return B.fdlb_diag(self.ctx)

    @property
    def tiling(self):
        return B.fdlb_get_tiling(self.ctx)

    def set_tiling(self, shape_id, group):
        B.fdlb_set_tiling(self.ctx, shape_id, group)

    def autotune(self, trial_steps=20, shape_ids=(), groups=(), cache=None):
        sizes = ",".join(f"{nx}x{ny}" for ny, nx in self.sizes)
        import hashlib
        key = f"{self.params[0].precision}:batch{len(self.sizes)}:" + hashlib.sha1(sizes.encode()).hexdigest()[:12]
        return _autotune(self, trial_steps, shape_ids, groups, cache, key=key)

    def close(self):
        if getattr(self, "ctx", None):
            B.fdlb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
