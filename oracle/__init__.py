"""CPU oracle for the stereographic-projection rotation vote.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the product path.  The compiled
part (aoresp_oracle.c) is plain single-threaded C built with
-O2 -ffp-contract=off; this module only marshals numpy arrays to it and adds a
few pure-numpy helpers used by the pins.

Parity status per function (see the module docstring of each test file for
the pins):
  coarse vote, fine vote, peak, top-k, axis, angle bin/histogram, rotation,
  inliers, least-squares rotation on the inlier set -- pinned (closed forms,
  brute force, invariants, noise-free recovery); end-to-end accuracy against
  the paper's reported error -- parity unpinned (the paper's figures are not
  recoverable).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "aoresp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fno-math-errno",
          "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-Wall"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (single-threaded, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Window(C.Structure):
    _fields_ = [("U0", C.c_float), ("V0", C.c_float), ("hx", C.c_float), ("hy", C.c_float),
                ("ix_lo", C.c_int), ("iy_lo", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
                ("M", C.c_int)]


class Result(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("axis", C.c_float * 3), ("angle", C.c_float),
                ("grid", C.c_uint32), ("peak_cell", C.c_uint32), ("fine_cell", C.c_uint32),
                ("angle_bin", C.c_uint32), ("axis_votes", C.c_uint32), ("fine_votes", C.c_uint32),
                ("angle_votes", C.c_uint32), ("n_inliers", C.c_uint32)]

    def todict(self) -> dict:
        return {
            "R": np.array(self.R[:], dtype=np.float32).reshape(3, 3),
            "axis": np.array(self.axis[:], dtype=np.float32),
            "angle": np.float32(self.angle),
            "grid": int(self.grid), "peak_cell": int(self.peak_cell),
            "fine_cell": int(self.fine_cell), "angle_bin": int(self.angle_bin),
            "axis_votes": int(self.axis_votes), "fine_votes": int(self.fine_votes),
            "angle_votes": int(self.angle_votes), "n_inliers": int(self.n_inliers),
        }


_lib = None
_f = C.c_float
_fp = C.POINTER(C.c_float)
_u32p = C.POINTER(C.c_uint32)
_u8p = C.POINTER(C.c_uint8)
_lp = C.POINTER(C.c_long)


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = C.CDLL(path)
        sig = {
            "or_displacement": (C.c_int, [_fp, _fp, _fp]),
            "or_coarse_coord": (_f, [C.c_int, C.c_int]),
            "or_W": (_f, [_f, _f]),
            "or_F": (_f, [_f, _f, _f, _f, _f, _f]),
            "or_coarse_hit": (C.c_int, [_fp, _fp, C.c_int, C.c_int, C.c_int]),
            "or_coarse_grid": (None, [_fp, _fp, C.c_long, C.c_int, _u32p]),
            "or_coarse_cell": (C.c_uint32, [_fp, _fp, C.c_long, C.c_int, C.c_int, C.c_int]),
            "or_arc_votes": (C.c_long, [_fp, _fp, C.c_int]),
            "or_argmax": (C.c_uint32, [_u32p, C.c_long, _lp]),
            "or_window_gate": (None, [_fp, _fp, C.c_long, C.c_int, C.c_int, C.c_int, C.c_int, _u8p]),
            "or_sample_dirs": (None, [C.c_int, _fp, _fp]),
            "or_sample_basis": (C.c_int, [_fp, _fp, _fp, _fp, _fp]),
            "or_sample_point": (None, [_fp, _fp, _f, _f, _fp]),
            "or_sample_cell": (C.c_long, [_fp, C.c_int]),
            "or_sample_grid": (None, [_fp, _fp, C.c_long, C.c_int, C.c_int, _u32p]),
            "or_fine_window": (None, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(Window)]),
            "or_fine_grid": (None, [_fp, _fp, C.c_long, C.POINTER(Window), _u32p]),
            "or_fine_cell": (C.c_uint32, [_fp, _fp, C.c_long, C.POINTER(Window), C.c_int, C.c_int]),
            "or_axis": (None, [_f, _f, _fp]),
            "or_coarse_center": (None, [C.c_int, C.c_int, C.c_int, _fp, _fp]),
            "or_fine_center": (None, [C.POINTER(Window), C.c_int, C.c_int, _fp, _fp]),
            "or_angle_xy": (None, [_fp, _fp, _fp, _fp, _fp]),
            "or_angle_boundaries": (None, [C.c_int, _fp, _fp]),
            "or_angle_centers": (None, [C.c_int, _fp, _fp, _fp]),
            "or_angle_bin": (C.c_int, [_fp, _fp, C.c_int, _f, _f]),
            "or_angle_hist": (None, [_fp, _fp, C.c_long, _fp, C.c_int, _u32p]),
            "or_rotation": (None, [_fp, _f, _f, _fp]),
            "or_inliers": (C.c_long, [_fp, _fp, _fp, C.c_long, _f, _u8p]),
            "or_rotation_error_deg": (C.c_double, [C.POINTER(C.c_double), _fp]),
            "or_suppressed": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
            "or_local_max": (C.c_int, [_u32p, C.c_int, C.c_int, C.c_int, C.c_int]),
            "or_topk_peaks": (C.c_int, [_u32p, C.c_int, C.c_int, C.c_int, _lp, _u32p]),
            "or_finish_peak": (None, [_fp, _fp, C.c_long, C.c_int, C.c_int, C.c_int, C.c_int, _f,
                                      C.c_long, C.c_uint32, C.POINTER(Result), _u8p, _u32p, _u32p]),
            "or_solve": (C.c_int, [_fp, _fp, C.c_long, C.c_int, C.c_int, C.c_int, C.c_int, _f,
                                   C.POINTER(Result), _u8p, _u32p, _u32p, _u32p]),
            "or_solve_topk": (C.c_int, [_fp, _fp, C.c_long, C.c_int, C.c_int, C.c_int, C.c_int, _f,
                                        C.c_int, C.c_int, C.POINTER(Result), _u8p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


# ----------------------------------------------------------------- scalar rule
def F(a, b, c, u, v, W) -> np.float32:
    return np.float32(lib().or_F(a, b, c, u, v, W))


def W(u, v) -> np.float32:
    return np.float32(lib().or_W(u, v))


def coarse_coord(G: int, j: int) -> np.float32:
    return np.float32(lib().or_coarse_coord(G, j))


def coarse_hit(p, q, G: int, ix: int, iy: int) -> bool:
    p, q = _f32(p), _f32(q)
    return bool(lib().or_coarse_hit(_ptr(p, _fp), _ptr(q, _fp), G, ix, iy))


# --------------------------------------------------------------- accumulators
def coarse_grid(P, Q, G: int) -> np.ndarray:
    P, Q = _f32(P), _f32(Q)
    n = P.shape[1]
    g = np.zeros(G * G, dtype=np.uint32)
    lib().or_coarse_grid(_ptr(P, _fp), _ptr(Q, _fp), n, G, _ptr(g, _u32p))
    return g.reshape(G, G)


def coarse_cell(P, Q, G: int, ix: int, iy: int) -> int:
    P, Q = _f32(P), _f32(Q)
    return int(lib().or_coarse_cell(_ptr(P, _fp), _ptr(Q, _fp), P.shape[1], G, ix, iy))


def arc_votes(p, q, G: int) -> int:
    p, q = _f32(p), _f32(q)
    return int(lib().or_arc_votes(_ptr(p, _fp), _ptr(q, _fp), G))


# ------------------------------------------------- literal sampling rule
def sample_dirs(J: int) -> tuple[np.ndarray, np.ndarray]:
    cs, sn = np.zeros(J, np.float32), np.zeros(J, np.float32)
    lib().or_sample_dirs(J, _ptr(cs, _fp), _ptr(sn, _fp))
    return cs, sn


def sample_basis(p, q):
    """(z, alpha1, alpha2) of Algorithm 1 for one correspondence, or None."""
    p, q = _f32(p), _f32(q)
    z, a1, a2 = (np.zeros(3, np.float32) for _ in range(3))
    ok = lib().or_sample_basis(_ptr(p, _fp), _ptr(q, _fp), _ptr(z, _fp), _ptr(a1, _fp), _ptr(a2, _fp))
    return (z, a1, a2) if ok else None


def sample_points(p, q, J: int) -> np.ndarray:
    """The J sample points of one correspondence's great circle, (3, J)."""
    b = sample_basis(p, q)
    if b is None:
        return np.zeros((3, 0), np.float32)
    _, a1, a2 = b
    cs, sn = sample_dirs(J)
    out = np.zeros((3, J), np.float32)
    s = np.zeros(3, np.float32)
    for j in range(J):
        lib().or_sample_point(_ptr(a1, _fp), _ptr(a2, _fp), cs[j], sn[j], _ptr(s, _fp))
        out[:, j] = s
    return out


def sample_cell(s, G: int) -> int:
    s = _f32(s)
    return int(lib().or_sample_cell(_ptr(s, _fp), G))


def sample_grid(P, Q, G: int, J: int) -> np.ndarray:
    """Coarse accumulator by the literal sampling rule (J samples per circle)."""
    P, Q = _f32(P), _f32(Q)
    g = np.zeros(G * G, dtype=np.uint32)
    lib().or_sample_grid(_ptr(P, _fp), _ptr(Q, _fp), P.shape[1], G, J, _ptr(g, _u32p))
    return g.reshape(G, G)


def argmax(a) -> tuple[int, int]:
    a = np.ascontiguousarray(a, dtype=np.uint32).ravel()
    idx = C.c_long(0)
    best = lib().or_argmax(_ptr(a, _u32p), a.size, C.byref(idx))
    return int(idx.value), int(best)


def fine_window(G: int, M: int, w: int, ix: int, iy: int) -> Window:
    win = Window()
    lib().or_fine_window(G, M, w, ix, iy, C.byref(win))
    return win


def fine_grid(P, Q, win: Window) -> np.ndarray:
    P, Q = _f32(P), _f32(Q)
    g = np.zeros(win.M * win.M, dtype=np.uint32)
    lib().or_fine_grid(_ptr(P, _fp), _ptr(Q, _fp), P.shape[1], C.byref(win), _ptr(g, _u32p))
    return g.reshape(win.M, win.M)


def fine_cell(P, Q, win: Window, jx: int, jy: int) -> int:
    P, Q = _f32(P), _f32(Q)
    return int(lib().or_fine_cell(_ptr(P, _fp), _ptr(Q, _fp), P.shape[1], C.byref(win), jx, jy))


# ------------------------------------------------------------ axis and angle
def axis(u, v) -> np.ndarray:
    r = np.zeros(3, dtype=np.float32)
    lib().or_axis(u, v, _ptr(r, _fp))
    return r


def coarse_center(G: int, ix: int, iy: int) -> tuple[np.float32, np.float32]:
    u, v = C.c_float(), C.c_float()
    lib().or_coarse_center(G, ix, iy, C.byref(u), C.byref(v))
    return np.float32(u.value), np.float32(v.value)


def fine_center(win: Window, jx: int, jy: int) -> tuple[np.float32, np.float32]:
    u, v = C.c_float(), C.c_float()
    lib().or_fine_center(C.byref(win), jx, jy, C.byref(u), C.byref(v))
    return np.float32(u.value), np.float32(v.value)


def angle_xy(r, p, q) -> tuple[np.float32, np.float32]:
    r, p, q = _f32(r), _f32(p), _f32(q)
    X, Y = C.c_float(), C.c_float()
    lib().or_angle_xy(_ptr(r, _fp), _ptr(p, _fp), _ptr(q, _fp), C.byref(X), C.byref(Y))
    return np.float32(X.value), np.float32(Y.value)


def angle_boundaries(B: int) -> tuple[np.ndarray, np.ndarray]:
    Tc = np.zeros(B, dtype=np.float32)
    Ts = np.zeros(B, dtype=np.float32)
    lib().or_angle_boundaries(B, _ptr(Tc, _fp), _ptr(Ts, _fp))
    return Tc, Ts


def angle_centers(B: int):
    th = np.zeros(B, dtype=np.float32)
    ct = np.zeros(B, dtype=np.float32)
    st = np.zeros(B, dtype=np.float32)
    lib().or_angle_centers(B, _ptr(th, _fp), _ptr(ct, _fp), _ptr(st, _fp))
    return th, ct, st


def angle_bin(Tc, Ts, X, Y) -> int:
    return int(lib().or_angle_bin(_ptr(Tc, _fp), _ptr(Ts, _fp), Tc.size, X, Y))


def angle_hist(P, Q, r, B: int) -> np.ndarray:
    P, Q, r = _f32(P), _f32(Q), _f32(r)
    h = np.zeros(B, dtype=np.uint32)
    lib().or_angle_hist(_ptr(P, _fp), _ptr(Q, _fp), P.shape[1], _ptr(r, _fp), B, _ptr(h, _u32p))
    return h


def rotation(r, ct, st) -> np.ndarray:
    r = _f32(r)
    R = np.zeros(9, dtype=np.float32)
    lib().or_rotation(_ptr(r, _fp), ct, st, _ptr(R, _fp))
    return R.reshape(3, 3)


def inliers(R, P, Q, tau: float) -> tuple[np.ndarray, int]:
    R, P, Q = _f32(R).ravel(), _f32(P), _f32(Q)
    n = P.shape[1]
    m = np.zeros(n, dtype=np.uint8)
    cnt = lib().or_inliers(_ptr(R, _fp), _ptr(P, _fp), _ptr(Q, _fp), n, tau, _ptr(m, _u8p))
    return m, int(cnt)


def rotation_error_deg(Rgt, R) -> float:
    Rgt = np.ascontiguousarray(Rgt, dtype=np.float64).ravel()
    R = _f32(R).ravel()
    return float(lib().or_rotation_error_deg(Rgt.ctypes.data_as(C.POINTER(C.c_double)), _ptr(R, _fp)))


def window_gate(P, Q, G: int, peak_cell: int, w: int) -> np.ndarray:
    """Correspondences whose curve votes for a cell of the (2w+1)^2 window of
    coarse cells around the peak (clipped), by the per-cell rule."""
    P, Q = _f32(P), _f32(Q)
    g = np.zeros(P.shape[1], dtype=np.uint8)
    lib().or_window_gate(_ptr(P, _fp), _ptr(Q, _fp), P.shape[1], G, peak_cell % G, peak_cell // G, w,
                         _ptr(g, _u8p))
    return g.astype(bool)


def angle_coarse_to_fine(P, Q, r, G: int, peak_cell: int, w: int, B: int, F: int, gate: bool = True) -> dict:
    """Coarse-to-fine angle voting (a variant of Sec. IV-B): only the
    correspondences that pass the window gate vote (all of them without the
    gate); the coarse B-bin histogram gives bin k (ties to the lowest bin);
    with F > 1 a second histogram over the partition of [-pi, pi) into B*F
    bins, read on the 3F fine bins of coarse bins k-1, k, k+1 (cyclically, in
    that order; ties to the first), gives the fine bin, and the angle and R
    come from that bin's centre (Eq. (2)); with F <= 1 from bin k's centre."""
    P, Q, r = _f32(P), _f32(Q), _f32(r)
    m = window_gate(P, Q, G, peak_cell, w) if gate else np.ones(P.shape[1], bool)
    Pg, Qg = np.ascontiguousarray(P[:, m]), np.ascontiguousarray(Q[:, m])
    h = angle_hist(Pg, Qg, r, B)
    k = int(np.argmax(h))
    out = {"gate": m, "hist": h, "angle_bin": k, "angle_votes": int(h[k]),
           "angle_fine_bin": 0, "angle_fine_votes": 0}
    if F <= 1:
        th, ct, st = angle_centers(B)
        out["angle"], out["R"] = np.float32(th[k]), rotation(r, ct[k], st[k])
        return out
    hf = angle_hist(Pg, Qg, r, B * F)
    win = [((k + dc) % B) * F + j for dc in (-1, 0, 1) for j in range(F)]
    vals = hf[win]
    jf = win[int(np.argmax(vals))]
    th, ct, st = angle_centers(B * F)
    out.update({"fine_hist": vals, "angle_fine_bin": jf, "angle_fine_votes": int(hf[jf]),
                "angle": np.float32(th[jf]), "R": rotation(r, ct[jf], st[jf])})
    return out


def ls_rotation(P, Q, mask) -> np.ndarray:
    """Least-squares rotation on an inlier set (a refinement step after the
    inlier test of Eq. (1); not part of the paper's Algorithm 1): the proper
    rotation R minimising sum over the set of ||R p_i - q_i||^2, in float64, by
    the SVD of H = sum p_i q_i^T (Kabsch): with H = U S V^T, R = V D U^T where
    D = diag(1, 1, sign det(V U^T)).  Fewer than three members: None."""
    P = np.asarray(P, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    m = np.asarray(mask).astype(bool)
    if int(m.sum()) < 3:
        return None
    H = P[:, m] @ Q[:, m].T
    U, _, Vt = np.linalg.svd(H)
    V = Vt.T
    d = 1.0 if np.linalg.det(V @ U.T) > 0 else -1.0
    return V @ np.diag([1.0, 1.0, d]) @ U.T


def suppressed(G: int, rad: int, px: int, py: int, ix: int, iy: int) -> bool:
    return bool(lib().or_suppressed(G, rad, px, py, ix, iy))


def local_max(grid, rad: int, ix: int, iy: int) -> bool:
    grid = np.ascontiguousarray(grid, dtype=np.uint32)
    return bool(lib().or_local_max(_ptr(grid.ravel(), _u32p), grid.shape[0], rad, ix, iy))


def topk_peaks(grid, k: int, rad: int):
    grid = np.ascontiguousarray(grid, dtype=np.uint32)
    G = grid.shape[0]
    peaks = np.zeros(k, dtype=np.int64)
    votes = np.zeros(k, dtype=np.uint32)
    pk = (C.c_long * k)()
    found = lib().or_topk_peaks(_ptr(grid.ravel(), _u32p), G, k, rad, pk, _ptr(votes, _u32p))
    peaks[:] = pk[:]
    return [(int(peaks[t]), int(votes[t])) for t in range(found)]


# ---------------------------------------------------------------- full solves
def finish_peak(P, Q, G, M, w, B, tau, peak, peak_votes, want_grids=False):
    P, Q = _f32(P), _f32(Q)
    n = P.shape[1]
    res = Result()
    mask = np.zeros(n, dtype=np.uint8)
    fine = np.zeros(max(M, 1) * max(M, 1), dtype=np.uint32)
    hist = np.zeros(B, dtype=np.uint32)
    lib().or_finish_peak(_ptr(P, _fp), _ptr(Q, _fp), n, G, M, w, B, tau, peak, peak_votes,
                         C.byref(res), _ptr(mask, _u8p), _ptr(fine, _u32p) if M > 0 else None,
                         _ptr(hist, _u32p))
    out = res.todict()
    out["mask"] = mask
    if want_grids:
        out["fine"] = fine.reshape(M, M) if M > 0 else None
        out["hist"] = hist
    return out


def solve(P, Q, G: int, B: int, M: int = 0, w: int = 1, tau: float = 0.05, want_grids: bool = False):
    P, Q = _f32(P), _f32(Q)
    n = P.shape[1]
    res = Result()
    mask = np.zeros(n, dtype=np.uint8)
    grid = np.zeros(G * G, dtype=np.uint32)
    fine = np.zeros(max(M, 1) * max(M, 1), dtype=np.uint32)
    hist = np.zeros(B, dtype=np.uint32)
    st = lib().or_solve(_ptr(P, _fp), _ptr(Q, _fp), n, G, M, w, B, tau, C.byref(res),
                        _ptr(mask, _u8p), _ptr(grid, _u32p),
                        _ptr(fine, _u32p) if M > 0 else None, _ptr(hist, _u32p))
    out = res.todict()
    out["status"] = int(st)
    out["mask"] = mask
    if want_grids:
        out["grid_full"] = grid.reshape(G, G)
        out["fine"] = fine.reshape(M, M) if M > 0 else None
        out["hist"] = hist
    return out


def solve_topk(P, Q, G: int, B: int, k: int, rad: int = 5, M: int = 0, w: int = 1, tau: float = 0.05):
    P, Q = _f32(P), _f32(Q)
    n = P.shape[1]
    res = (Result * k)()
    masks = np.zeros(k * n, dtype=np.uint8)
    found = lib().or_solve_topk(_ptr(P, _fp), _ptr(Q, _fp), n, G, M, w, B, tau, k, rad, res,
                                _ptr(masks, _u8p))
    out = []
    for t in range(found):
        d = res[t].todict()
        d["mask"] = masks[t * n:(t + 1) * n].copy()
        out.append(d)
    return out


if __name__ == "__main__":  # pragma: no cover
    build(force=True)
    print("built", _LIB, file=sys.stderr)
