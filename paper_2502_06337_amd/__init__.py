"""paper_2502_06337_amd: outlier-robust rotation estimation by stereographic
projection and spatial voting (Xu, Liu, Wang, Yang, arXiv 2502.06337) on
AMD Instinct MI355X.

The estimation runs in libaoresp.so (HIP kernels for gfx950 behind a C ABI,
include/aoresp.h).  This package is a thin binding with the same names:

  est_rotation(P, Q, params)            one rotation (Algorithm 1)
  est_rotations_topk(P, Q, k, params)   several rotations (Sec. IV-D)
  est_rotation_batch(Ps, Qs, params)    many independent instances, batched
  coarse_grid(P, Q, G)                  the axis accumulator (device tensors)
  solve_debug(P, Q, params)             a solve plus its accumulators
  autotune(P, Q, params)                pick the coarse vote's work split for (G, n)
  Server                                 request loop with continuous batching

P and Q are (3, n) float32: numpy arrays (host entry points) or torch CUDA
tensors (device entry points, torch's current stream).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (AorespError, Params, Result, ServerCfg, SolveParams, EBUSY, EDEVICE, EINVAL, ENODATA,
                   ENOMEM, ETIMEDOUT, OK)

__all__ = ["est_rotation", "est_rotations_topk", "est_rotation_batch", "coarse_grid", "solve_debug",
           "grid_for_n", "autotune", "tuner_get", "tuner_save", "tuner_load", "tuner_clear", "Server",
           "SolveParams", "AorespError", "load_library"]


def load_library():
    return _lib.load()


def grid_for_n(n: int) -> int:
    return int(_lib.load().aoresp_grid_for_n(int(n)))


def _vp(x) -> int | None:
    if x is None:
        return None
    if _lib._is_torch(x):
        return int(x.data_ptr())
    return x.ctypes.data


def est_rotation(P, Q, params=None, want_mask: bool = True):
    """Single rotation.  Returns (result dict, mask or None, status)."""
    L = _lib.load()
    prm = _lib._params(params)
    res = Result()
    P, Q = _lib._pair(P, Q)
    if _lib._is_torch(P):
        import torch
        n = P.shape[1]
        mask = torch.empty(n, dtype=torch.uint8, device=P.device) if want_mask else None
        st = L.est_rotation_dev(_vp(P), _vp(Q), n, C.byref(prm), C.byref(res), _vp(mask), _lib._stream_ptr(P))
    else:
        n = P.shape[1]
        mask = np.empty(n, dtype=np.uint8) if want_mask else None
        st = L.est_rotation(_vp(P), _vp(Q), n, C.byref(prm), C.byref(res), _vp(mask))
    _lib._check(st, "est_rotation")
    return res.todict(), mask, st


def est_rotations_topk(P, Q, k: int, params=None, want_mask: bool = True):
    """Several rotations.  Returns (list of result dicts, masks (k, n) or None, status)."""
    L = _lib.load()
    prm = _lib._params(params)
    res = (Result * k)()
    found = C.c_uint32(0)
    P, Q = _lib._pair(P, Q)
    if _lib._is_torch(P):
        import torch
        n = P.shape[1]
        masks = torch.empty((k, n), dtype=torch.uint8, device=P.device) if want_mask else None
        st = L.est_rotations_topk_dev(_vp(P), _vp(Q), n, k, C.byref(prm), res, _vp(masks), C.byref(found),
                                      _lib._stream_ptr(P))
    else:
        n = P.shape[1]
        masks = np.empty((k, n), dtype=np.uint8) if want_mask else None
        st = L.est_rotations_topk(_vp(P), _vp(Q), n, k, C.byref(prm), res, _vp(masks), C.byref(found))
    _lib._check(st, "est_rotations_topk")
    nf = int(found.value)
    return [res[t].todict() for t in range(nf)], (masks[:nf] if masks is not None else None), st


def est_rotation_batch(P, Q, offsets, params=None, want_mask: bool = True):
    """Batched instances.  P, Q: (3, N) concatenated columns; offsets: batch+1
    column offsets.  params: one entry or a list with one per instance.
    Returns (list of result dicts, mask (N,) or None, status)."""
    L = _lib.load()
    P, Q = _lib._pair(P, Q)
    off = _lib._offsets(offsets, P.shape[1])
    batch = off.size - 1
    if isinstance(params, (list, tuple)):
        prm_arr = (Params * len(params))(*[_lib._params(p) for p in params])
        pc = len(params)
    else:
        prm_arr = (Params * 1)(_lib._params(params))
        pc = 1
    res = (Result * max(batch, 1))()
    if _lib._is_torch(P):
        import torch
        N = P.shape[1]
        mask = torch.empty(N, dtype=torch.uint8, device=P.device) if want_mask else None
        st = L.est_rotation_batch_dev(_vp(P), _vp(Q), off.ctypes.data, batch, prm_arr, pc, res, _vp(mask),
                                      _lib._stream_ptr(P))
    else:
        N = P.shape[1]
        mask = np.empty(N, dtype=np.uint8) if want_mask else None
        st = L.est_rotation_batch(_vp(P), _vp(Q), off.ctypes.data, batch, prm_arr, pc, res, _vp(mask))
    _lib._check(st, "est_rotation_batch")
    return [res[b].todict() for b in range(batch)], mask, st


def coarse_grid(P, Q, G: int):
    """Axis accumulator of device tensors P, Q: (G, G) uint32 torch tensor (int32 view)."""
    import torch
    L = _lib.load()
    P, Q = _lib._pair(P, Q)
    if not _lib._is_torch(P):
        raise ValueError("coarse_grid takes torch CUDA tensors")
    grid = torch.empty((G, G), dtype=torch.int32, device=P.device)
    st = L.aoresp_coarse_grid_dev(_vp(P), _vp(Q), P.shape[1], G, _vp(grid), _lib._stream_ptr(P))
    _lib._check(st, "aoresp_coarse_grid_dev", allow=(OK,))
    return grid


def solve_debug(P, Q, params=None):
    """Single solve on device tensors, returning the accumulators as well."""
    import torch
    L = _lib.load()
    prm = _lib._params(params)
    P, Q = _lib._pair(P, Q)
    if not _lib._is_torch(P):
        raise ValueError("solve_debug takes torch CUDA tensors")
    n = P.shape[1]
    G = prm.grid or grid_for_n(n)
    M = prm.refine_grid
    B = prm.angle_bins or 360
    grid = torch.zeros((G, G), dtype=torch.int32, device=P.device)
    fine = torch.zeros((M, M), dtype=torch.int32, device=P.device) if M else None
    hist = torch.zeros(B, dtype=torch.int32, device=P.device)
    mask = torch.empty(n, dtype=torch.uint8, device=P.device)
    res = Result()
    st = L.aoresp_solve_debug_dev(_vp(P), _vp(Q), n, C.byref(prm), C.byref(res), _vp(mask), _vp(grid),
                                  _vp(fine), _vp(hist), _lib._stream_ptr(P))
    _lib._check(st, "aoresp_solve_debug_dev")
    return {"result": res.todict(), "mask": mask, "grid": grid, "fine": fine, "hist": hist, "status": st}


class Server:
    """Request loop: submit() copies a problem and returns an id; poll() returns
    (status, result dict, mask) once it is done."""

    def __init__(self, hbm_budget_bytes: int = 0, max_slots: int = 0, timeout_us: int = 0):
        L = _lib.load()
        cfg = ServerCfg(hbm_budget_bytes, max_slots, timeout_us)
        h = C.c_void_p()
        _lib._check(L.aoresp_server_create(C.byref(cfg), C.byref(h)), "aoresp_server_create", allow=(OK,))
        self._h = h
        self._n = {}

    def submit(self, P, Q, params=None) -> int:
        L = _lib.load()
        P, Q = _lib._pair(P, Q)
        if _lib._is_torch(P):
            raise ValueError("Server.submit takes host (numpy) arrays")
        prm = _lib._params(params)
        rid = C.c_uint64(0)
        _lib._check(L.aoresp_submit(self._h, P.ctypes.data, Q.ctypes.data, P.shape[1], C.byref(prm),
                                    C.byref(rid)), "aoresp_submit", allow=(OK,))
        self._n[int(rid.value)] = P.shape[1]
        return int(rid.value)

    def poll(self, rid: int, timeout_us: int = -1, want_mask: bool = True):
        L = _lib.load()
        res = Result()
        n = self._n.get(rid, 0)
        mask = np.empty(max(n, 1), dtype=np.uint8) if want_mask else None
        st = L.aoresp_poll(self._h, rid, C.byref(res), _vp(mask), timeout_us)
        if st == EBUSY:
            return st, None, None
        self._n.pop(rid, None)
        if st not in (OK, ENODATA):
            return st, None, None
        return st, res.todict(), (mask[:n] if mask is not None else None)

    def stats(self) -> dict:
        L = _lib.load()
        p50, p99, rps = C.c_double(), C.c_double(), C.c_double()
        done = C.c_uint64()
        L.aoresp_server_stats(self._h, C.byref(p50), C.byref(p99), C.byref(rps), C.byref(done))
        return {"p50_us": p50.value, "p99_us": p99.value, "req_per_s": rps.value, "completed": done.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().aoresp_server_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def autotune(P, Q, params=None) -> dict:
    """Time the coarse vote of a solve of (P, Q) (torch CUDA tensors) under
    each candidate work split and keep the fastest for (G, n bucket).  Results
    of later solves are unchanged (bit-identical); only their speed is."""
    L = _lib.load()
    prm = _lib._params(params)
    P, Q = _lib._pair(P, Q)
    if not _lib._is_torch(P):
        raise ValueError("autotune takes torch CUDA tensors")
    out = _lib.Tuning()
    st = L.aoresp_autotune_dev(_vp(P), _vp(Q), P.shape[1], C.byref(prm), C.byref(out), _lib._stream_ptr(P))
    if st != OK:
        raise AorespError(st, "aoresp_autotune_dev")
    return out.todict()


def tuner_get(grid: int, n: int) -> dict:
    out = _lib.Tuning()
    st = _lib.load().aoresp_tuner_get(int(grid), int(n), C.byref(out))
    if st != OK:
        raise AorespError(st, "aoresp_tuner_get")
    return out.todict()


def tuner_save(path: str) -> None:
    st = _lib.load().aoresp_tuner_save(path.encode())
    if st != OK:
        raise AorespError(st, "aoresp_tuner_save")


def tuner_load(path: str) -> None:
    st = _lib.load().aoresp_tuner_load(path.encode())
    if st != OK:
        raise AorespError(st, "aoresp_tuner_load")


def tuner_clear() -> None:
    st = _lib.load().aoresp_tuner_clear()
    if st != OK:
        raise AorespError(st, "aoresp_tuner_clear")
