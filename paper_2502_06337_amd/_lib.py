"""ctypes binding of libaoresp.so (include/aoresp.h).

Argument marshalling only: every step of the estimation runs in the HIP
library.  Host arrays (numpy) go to the host entry points; torch CUDA tensors
go to the *_dev entry points on torch's current stream.  There is no CPU
fallback: if the library is missing the import of any entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaoresp.so")

OK, EINVAL, ENOMEM, EDEVICE, ENODATA, EBUSY, ETIMEDOUT = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENODATA", -5: "EBUSY",
                -6: "ETIMEDOUT"}


class AorespError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("grid", C.c_uint32), ("refine_grid", C.c_uint32), ("refine_halfwin", C.c_uint32),
                ("angle_bins", C.c_uint32), ("nms_radius", C.c_uint32), ("inlier_thresh", C.c_float),
                ("angle_gate", C.c_uint32), ("angle_refine", C.c_uint32), ("vote_rule", C.c_uint32),
                ("circle_samples", C.c_uint32)]


class Result(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("axis", C.c_float * 3), ("angle", C.c_float),
                ("grid", C.c_uint32), ("peak_cell", C.c_uint32), ("fine_cell", C.c_uint32),
                ("angle_bin", C.c_uint32), ("axis_votes", C.c_uint32), ("fine_votes", C.c_uint32),
                ("angle_votes", C.c_uint32), ("n_inliers", C.c_uint32), ("R_ls", C.c_float * 9),
                ("angle_fine_bin", C.c_uint32), ("angle_fine_votes", C.c_uint32)]

    def todict(self) -> dict:
        return {
            "R": np.array(self.R[:], dtype=np.float32).reshape(3, 3),
            "axis": np.array(self.axis[:], dtype=np.float32),
            "angle": np.float32(self.angle),
            "grid": int(self.grid), "peak_cell": int(self.peak_cell), "fine_cell": int(self.fine_cell),
            "angle_bin": int(self.angle_bin), "axis_votes": int(self.axis_votes),
            "fine_votes": int(self.fine_votes), "angle_votes": int(self.angle_votes),
            "n_inliers": int(self.n_inliers),
            "R_ls": np.array(self.R_ls[:], dtype=np.float32).reshape(3, 3),
            "angle_fine_bin": int(self.angle_fine_bin), "angle_fine_votes": int(self.angle_fine_votes),
        }


class Tuning(C.Structure):
    _fields_ = [("grid", C.c_uint32), ("n_bucket", C.c_uint32), ("tile_cells", C.c_uint32),
                ("vote_target", C.c_float), ("vote_ms", C.c_float)]

    def todict(self) -> dict:
        return {"grid": int(self.grid), "n_bucket": int(self.n_bucket), "tile_cells": int(self.tile_cells),
                "vote_target": float(self.vote_target), "vote_ms": float(self.vote_ms)}


class ServerCfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_uint32), ("timeout_us", C.c_uint32)]


# every symbol the header declares, with its signature
_vp, _fp, _u8p, _u32p, _u64p = C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p
SIGNATURES = {
    "aoresp_grid_for_n": (C.c_uint32, [C.c_uint64]),
    "est_rotation": (C.c_int, [_fp, _fp, C.c_size_t, C.POINTER(Params), C.POINTER(Result), _u8p]),
    "est_rotation_dev": (C.c_int, [_fp, _fp, C.c_size_t, C.POINTER(Params), C.POINTER(Result), _u8p, _vp]),
    "est_rotation_noalloc_dev": (C.c_int, [_fp, _fp, C.c_size_t, C.POINTER(Params), C.POINTER(Result), _u8p,
                                           _vp]),
    "est_rotations_topk": (C.c_int, [_fp, _fp, C.c_size_t, C.c_uint32, C.POINTER(Params), C.POINTER(Result),
                                     _u8p, C.POINTER(C.c_uint32)]),
    "est_rotations_topk_dev": (C.c_int, [_fp, _fp, C.c_size_t, C.c_uint32, C.POINTER(Params),
                                         C.POINTER(Result), _u8p, C.POINTER(C.c_uint32), _vp]),
    "est_rotation_batch": (C.c_int, [_fp, _fp, _u64p, C.c_uint32, C.POINTER(Params), C.c_uint32,
                                     C.POINTER(Result), _u8p]),
    "est_rotation_batch_dev": (C.c_int, [_fp, _fp, _u64p, C.c_uint32, C.POINTER(Params), C.c_uint32,
                                         C.POINTER(Result), _u8p, _vp]),
    "aoresp_coarse_grid_dev": (C.c_int, [_fp, _fp, C.c_size_t, C.c_uint32, _u32p, _vp]),
    "aoresp_solve_debug_dev": (C.c_int, [_fp, _fp, C.c_size_t, C.POINTER(Params), C.POINTER(Result), _u8p,
                                         _u32p, _u32p, _u32p, _vp]),
    "aoresp_stage_times_dev": (C.c_int, [_fp, _fp, C.c_size_t, C.POINTER(Params), C.POINTER(C.c_float),
                                         C.POINTER(C.c_uint32), _vp]),
    "aoresp_autotune_dev": (C.c_int, [_fp, _fp, C.c_size_t, C.POINTER(Params), C.POINTER(Tuning), _vp]),
    "aoresp_tuner_get": (C.c_int, [C.c_uint32, C.c_uint64, C.POINTER(Tuning)]),
    "aoresp_tuner_save": (C.c_int, [C.c_char_p]),
    "aoresp_tuner_load": (C.c_int, [C.c_char_p]),
    "aoresp_tuner_clear": (C.c_int, []),
    "aoresp_server_create": (C.c_int, [C.POINTER(ServerCfg), C.POINTER(C.c_void_p)]),
    "aoresp_submit": (C.c_int, [_vp, _fp, _fp, C.c_size_t, C.POINTER(Params), C.POINTER(C.c_uint64)]),
    "aoresp_poll": (C.c_int, [_vp, C.c_uint64, C.POINTER(Result), _u8p, C.c_int64]),
    "aoresp_server_stats": (C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "aoresp_server_destroy": (None, [_vp]),
    "aoresp_strerror": (C.c_char_p, [C.c_int]),
    "aoresp_version": (C.c_char_p, []),
}

_lib = None


def load(path: str | None = None):
    """Load the in-tree libaoresp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"libaoresp.so not built at {path}; run paper_2502_06337_amd/build.py")
    L = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


@dataclass
class SolveParams:
    grid: int = 0
    refine_grid: int = 0
    refine_halfwin: int = 0
    angle_bins: int = 0
    nms_radius: int = 0
    inlier_thresh: float = 0.0
    angle_gate: int = 0
    angle_refine: int = 0
    vote_rule: int = 0
    circle_samples: int = 0

    def c(self) -> Params:
        return Params(self.grid, self.refine_grid, self.refine_halfwin, self.angle_bins, self.nms_radius,
                      self.inlier_thresh, self.angle_gate, self.angle_refine, self.vote_rule, self.circle_samples)


def _params(prm) -> Params:
    if prm is None:
        return Params()
    if isinstance(prm, Params):
        return prm
    if isinstance(prm, SolveParams):
        return prm.c()
    if isinstance(prm, dict):
        return SolveParams(**prm).c()
    raise TypeError("params must be SolveParams, dict or Params")


def _check(st: int, what: str, allow=(OK, ENODATA)) -> int:
    if st not in allow:
        raise AorespError(st, what)
    return st


def _is_torch(x) -> bool:
    try:
        import torch
        return isinstance(x, torch.Tensor)
    except ImportError:  # pragma: no cover
        return False


def _stream_ptr(dev_tensor) -> int:
    import torch
    return int(torch.cuda.current_stream(dev_tensor.device).cuda_stream)


def _host_soa(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim != 2 or a.shape[0] != 3:
        raise ValueError("expected a (3, n) float32 array")
    return a


def _dev_soa(t):
    import torch
    if t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] != 3 or not t.is_cuda:
        raise ValueError("expected a (3, n) float32 CUDA tensor")
    return t.contiguous()


def _pair(P, Q):
    """P and Q as one host pair or one device pair of equal (3, n) shape: the
    library reads n columns of both, so a shorter Q would be read past its
    end."""
    if _is_torch(P) != _is_torch(Q):
        raise ValueError("P and Q must both be numpy arrays or both be torch tensors")
    if _is_torch(P):
        P, Q = _dev_soa(P), _dev_soa(Q)
        if P.device != Q.device:
            raise ValueError(f"P and Q are on different devices ({P.device}, {Q.device})")
    else:
        P, Q = _host_soa(P), _host_soa(Q)
    if P.shape != Q.shape:
        raise ValueError(f"P and Q must have the same shape, got {tuple(P.shape)} and {tuple(Q.shape)}")
    return P, Q


def _offsets(offsets, ncols: int) -> np.ndarray:
    """Batch column offsets: batch + 1 non-decreasing entries from 0 to the
    number of columns of P and Q."""
    off = np.asarray(offsets)
    if off.ndim != 1 or off.size < 2:
        raise ValueError("offsets must be a 1-D sequence of batch + 1 column offsets")
    if not np.issubdtype(off.dtype, np.integer):
        raise ValueError("offsets must be integers")
    if int(off[0]) != 0 or int(off[-1]) != int(ncols):
        raise ValueError(f"offsets must run from 0 to {ncols} (the columns of P and Q), got "
                         f"{int(off[0])} .. {int(off[-1])}")
    if (np.diff(off.astype(np.int64)) < 0).any():
        raise ValueError("offsets must not decrease")
    return np.ascontiguousarray(off, dtype=np.uint64)
