"""Host-side checks that need no GPU: the binding refuses to run without the
HIP library (no CPU fallback), the seeded generator is deterministic and
shaped as stated, and the benchmark refuses more than one GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2502_06337_amd import _lib, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_binding_fails_loudly_without_library(tmp_path):
    saved = _lib._lib
    _lib._lib = None
    try:
        with pytest.raises(ImportError):
            _lib.load(str(tmp_path / "missing" / "libaoresp.so"))
    finally:
        _lib._lib = saved


def test_generator_is_deterministic_and_shaped():
    a = synth.make_instance(5000, 123, outlier_rate=0.9, sigma=0.01)
    b = synth.make_instance(5000, 123, outlier_rate=0.9, sigma=0.01)
    c = synth.make_instance(5000, 124, outlier_rate=0.9, sigma=0.01)
    assert a.P.dtype == np.float32 and a.P.shape == (3, 5000) and a.Q.shape == (3, 5000)
    assert np.array_equal(a.P, b.P) and np.array_equal(a.Q, b.Q)
    assert not np.array_equal(a.P, c.P)
    assert (a.P >= -1).all() and (a.P < 1).all()
    # 10% inliers: q = R p + noise, residual about sigma * sqrt(3)
    R = np.asarray(a.R_gt[0], dtype=np.float64)
    res = np.linalg.norm(R @ a.P.astype(np.float64) - a.Q.astype(np.float64), axis=0)
    inl = res < 0.1
    assert abs(int(inl.sum()) - 500) <= 5
    assert 0.005 < float(np.median(res[inl])) < 0.03
    # inliers are not contiguous (permuted indices)
    idx = np.flatnonzero(inl)
    assert idx.max() - idx.min() > 2000


def test_generator_rotation_is_proper():
    for s in range(20):
        R = synth.random_rotation(s)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(R) - 1.0) < 1e-12


def test_multi_rotation_instance():
    inst = synth.make_instance(3000, 7, n_rot=3, inlier_frac_each=0.1, sigma=0.0)
    assert len(inst.R_gt) == 3
    P, Q = inst.P.astype(np.float64), inst.Q.astype(np.float64)
    for R in inst.R_gt:
        exact = np.linalg.norm(np.asarray(R) @ P - Q, axis=0) < 1e-5
        assert abs(int(exact.sum()) - 300) <= 3


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_binding_rejects_mismatched_inputs():
    """Shapes, kinds and batch offsets are checked before any call into the
    library: n comes from P, so a shorter Q would be read past its end."""
    import paper_2502_06337_amd as aor
    P = np.zeros((3, 10), dtype=np.float32)
    with pytest.raises(ValueError, match="same shape"):
        aor.est_rotation(P, np.zeros((3, 9), dtype=np.float32))
    with pytest.raises(ValueError, match="same shape"):
        aor.est_rotations_topk(P, np.zeros((3, 11), dtype=np.float32), 2)
    with pytest.raises(ValueError, match="same shape"):
        aor.est_rotation_batch(P, np.zeros((3, 9), dtype=np.float32), [0, 5, 10])
    with pytest.raises(ValueError, match=r"\(3, n\)"):
        aor.est_rotation(np.zeros((4, 10), dtype=np.float32), np.zeros((4, 10), dtype=np.float32))
    torch = pytest.importorskip("torch")
    with pytest.raises(ValueError, match="both"):
        aor.est_rotation(P, torch.zeros((3, 10), dtype=torch.float32))
    with pytest.raises(ValueError, match="CUDA"):
        aor.est_rotation(torch.zeros((3, 10)), torch.zeros((3, 10)))


def test_binding_rejects_bad_batch_offsets():
    import paper_2502_06337_amd as aor
    P = np.zeros((3, 10), dtype=np.float32)
    Q = np.zeros((3, 10), dtype=np.float32)
    with pytest.raises(ValueError, match="run from 0 to 10"):
        aor.est_rotation_batch(P, Q, [0, 5, 9])       # total below the columns
    with pytest.raises(ValueError, match="run from 0 to 10"):
        aor.est_rotation_batch(P, Q, [0, 5, 12])      # total beyond them
    with pytest.raises(ValueError, match="run from 0 to 10"):
        aor.est_rotation_batch(P, Q, [1, 5, 10])
    with pytest.raises(ValueError, match="not decrease"):
        aor.est_rotation_batch(P, Q, [0, 7, 3, 10])
    with pytest.raises(ValueError, match="integers"):
        aor.est_rotation_batch(P, Q, [0.0, 10.0])
    with pytest.raises(ValueError, match="batch"):
        aor.est_rotation_batch(P, Q, [10])
