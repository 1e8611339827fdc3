"""The library's octant pieces and line walks, built for the host
(tests/host_walk.hip), against the oracle on the CPU: coarse and refinement
accumulators bit-exact on seeded and adversarial correspondences, and an audit
of every clean line of the certified walk (the two vertex signs its
certificates vouch for are evaluated and must agree)."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2502_06337_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def hw(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("hostwalk") / "libhostwalk.so")
    cmd = [hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-x", "hip",
           os.path.join(HERE, "host_walk.hip"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    lib = C.CDLL(out)
    for fn in (lib.hw_coarse_grid, lib.hw_fine_grid):
        fn.restype = C.c_int
    lib.hw_coarse_grid.argtypes = [C.c_void_p, C.c_void_p, C.c_long, C.c_int, C.c_void_p, C.c_void_p]
    lib.hw_fine_grid.argtypes = [C.c_void_p, C.c_void_p, C.c_long, C.c_float, C.c_float, C.c_float, C.c_float,
                                 C.c_int, C.c_void_p, C.c_void_p]
    return lib


def host_coarse(hw, P, Q, G):
    P = np.ascontiguousarray(P, np.float32)
    Q = np.ascontiguousarray(Q, np.float32)
    g = np.zeros(G * G, np.uint32)
    audit = np.zeros(2, np.int64)
    bad = hw.hw_coarse_grid(P.ctypes.data, Q.ctypes.data, P.shape[1], G, g.ctypes.data, audit.ctypes.data)
    return g.reshape(G, G), bad, audit


def host_fine(hw, P, Q, win):
    P = np.ascontiguousarray(P, np.float32)
    Q = np.ascontiguousarray(Q, np.float32)
    g = np.zeros(win.M * win.M, np.uint32)
    audit = np.zeros(2, np.int64)
    bad = hw.hw_fine_grid(P.ctypes.data, Q.ctypes.data, P.shape[1], win.U0, win.V0, win.hx, win.hy, win.M,
                          g.ctypes.data, audit.ctypes.data)
    return g.reshape(win.M, win.M), bad, audit


def adversarial(rng, n):
    """Displacements near the walk's special cases: tiny or zero c (near-lines
    and lines), slope-one octants, magnitudes outside the walk's range
    (exhaustive path), axis-aligned and degenerate ones."""
    D = rng.uniform(-1, 1, (3, n))
    k = rng.integers(0, 8, n)
    D[2, k == 0] *= 1e-6
    D[2, k == 1] = 0.0
    D[0, k == 2] = D[1, k == 2] * (1 + rng.uniform(-1e-6, 1e-6, int((k == 2).sum())))
    D[:, k == 3] *= 1e-20
    D[2, k == 4] = 1e-30
    D[0, k == 5] = 0.0
    D[:, k == 6] = 0.0
    return D.astype(np.float32)


@pytest.mark.parametrize("G,n,seed", [(64, 600, 1), (256, 400, 2), (1024, 250, 3)])
def test_coarse_walk_matches_oracle(hw, orc, G, n, seed):
    inst = synth.make_instance(n, seed, outlier_rate=0.9, sigma=0.01)
    g, bad, audit = host_coarse(hw, inst.P, inst.Q, G)
    assert bad == 0
    assert np.array_equal(g, orc.coarse_grid(inst.P, inst.Q, G))
    assert audit[0] > 0 and audit[1] == 0


@pytest.mark.parametrize("G", [64, 128, 512])
def test_coarse_walk_adversarial(hw, orc, G):
    rng = np.random.default_rng(100 + G)
    D = adversarial(rng, 400)
    Z = np.zeros_like(D)
    g, bad, audit = host_coarse(hw, D, Z, G)
    assert bad == 0
    assert np.array_equal(g, orc.coarse_grid(D, Z, G))
    assert audit[1] == 0


def test_fine_walk_matches_oracle(hw, orc):
    rng = np.random.default_rng(7)
    done = 0
    for _ in range(40):
        G = int(rng.choice([128, 256, 1024]))
        M = int(rng.choice([16, 32, 64]))
        ix, iy = (int(v) for v in rng.integers(0, G, 2))
        win = orc.fine_window(G, M, 1, ix, iy)
        if win.U0 ** 2 + win.V0 ** 2 > 1.2:
            continue
        # great circles through the axis of the window centre, plus adversarial ones
        uc, vc = win.U0 + win.hx * M / 2, win.V0 + win.hy * M / 2
        s = uc * uc + vc * vc
        r0 = np.array([2 * uc / (1 + s), 2 * vc / (1 + s), (s - 1) / (1 + s)])
        D1 = np.cross(r0[None, :], rng.normal(size=(120, 3))).T
        D = np.concatenate([D1, adversarial(rng, 120)], axis=1).astype(np.float32)
        Z = np.zeros_like(D)
        f, bad, audit = host_fine(hw, D, Z, win)
        assert bad == 0, (G, M, ix, iy)
        assert np.array_equal(f, orc.fine_grid(D, Z, win)), (G, M, ix, iy)
        assert audit[1] == 0
        done += 1
    assert done >= 15


@pytest.mark.parametrize("G", [64, 1024])
def test_certificate_audit_at_scale(hw, G):
    """1e5 correspondences of the benchmark's distribution: every clean line's
    neighbouring rows have the signs the certificates claim (about 1.2e8 lines
    at G = 1024)."""
    inst = synth.make_instance(100_000, 2000, outlier_rate=0.9, sigma=0.01)
    g, bad, audit = host_coarse(hw, inst.P, inst.Q, G)
    assert bad == 0
    assert audit[0] > (1e8 if G == 1024 else 5e6)
    assert audit[1] == 0


@pytest.mark.parametrize("G", [128, 4096])
def test_clean_cells_within_bounds(hw, G):
    """Uniformly oriented great circles and adversarial ones: no clean line of
    a certified walk counts a cell past its row quarter's column bound or
    beyond the tile's pad words (the kernel writes those cells unchecked), and
    every fast value beyond the threshold has the rule's sign."""
    rng = np.random.default_rng(31 + G)
    D = np.concatenate([rng.normal(size=(3, 3000)), adversarial(rng, 1000)], axis=1).astype(np.float32)
    Z = np.zeros_like(D)
    g, bad, audit = host_coarse(hw, D, Z, G)
    assert bad == 0
    assert audit[0] > 1e6 and audit[1] == 0


def test_ls_rotation_solve_matches_oracle(hw, orc):
    """The library's quaternion solve (host build) against the oracle's SVD
    solve on the same float64 sums: equal to a few float32 rounding steps."""
    hw.hw_ls_rotation.restype = None
    hw.hw_ls_rotation.argtypes = [C.c_void_p, C.c_void_p]
    rng = np.random.default_rng(21)
    for trial in range(200):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        n = int(rng.integers(3, 200))
        P = rng.uniform(-1, 1, (3, n)).astype(np.float32)
        Q = (R @ P + rng.uniform(0.0, 0.05) * rng.normal(size=(3, n))).astype(np.float32)
        m = np.ones(n, bool)
        S = np.ascontiguousarray((P.astype(np.float64) @ Q.astype(np.float64).T).ravel())
        out = np.zeros(9, np.float32)
        hw.hw_ls_rotation(S.ctypes.data, out.ctypes.data)
        ref = orc.ls_rotation(P, Q, m)
        assert np.max(np.abs(out.reshape(3, 3).astype(np.float64) - ref)) <= 2.0 ** -22, trial
