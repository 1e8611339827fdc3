"""The allocation-free entry point (est_rotation_noalloc_dev) through the C
ABI: bit-identical to est_rotation_dev (result, least-squares rotation and
mask) on two calls in a row, the second smaller than the first, with and
without refinement and with the sampling rule; a solve that does not fit its static scratch array is
refused with ENOMEM before anything runs."""
import ctypes as C

import numpy as np
import pytest

from paper_2502_06337_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_06337_amd as aor
    return aor.load_library()


def solve(L, fn, P, Q, prm):
    from paper_2502_06337_amd import _lib
    n = P.shape[1]
    res = _lib.Result()
    mask = torch.full((n,), 7, dtype=torch.uint8, device=P.device)
    st = getattr(L, fn)(P.data_ptr(), Q.data_ptr(), n, C.byref(_lib._params(prm)), C.byref(res), mask.data_ptr(),
                        torch.cuda.current_stream(P.device).cuda_stream)
    torch.cuda.synchronize()
    return st, res.todict(), mask.cpu().numpy()


def assert_same(a, b):
    sa, ra, ma = a
    sb, rb, mb = b
    assert sa == sb
    for k in ("peak_cell", "axis_votes", "fine_cell", "fine_votes", "angle_bin", "angle_votes", "n_inliers", "grid"):
        assert ra[k] == rb[k], (k, ra[k], rb[k])
    for k in ("axis", "R", "R_ls"):
        assert np.array_equal(np.asarray(ra[k], np.float32).view(np.uint32),
                              np.asarray(rb[k], np.float32).view(np.uint32)), k
    assert np.float32(ra["angle"]).view(np.uint32) == np.float32(rb["angle"]).view(np.uint32)
    assert np.array_equal(ma, mb)


@pytest.mark.parametrize("M", [0, 64])
def test_noalloc_equals_est_rotation_dev(lib, M):
    from paper_2502_06337_amd import SolveParams
    for n, seed in ((300000, 61), (20000, 62)):   # second call smaller than the first
        inst = synth.make_instance(n, seed, outlier_rate=0.9)
        P = torch.from_numpy(inst.P).cuda()
        Q = torch.from_numpy(inst.Q).cuda()
        prm = SolveParams(refine_grid=M, angle_bins=3600 if M else 360)
        got = solve(lib, "est_rotation_noalloc_dev", P, Q, prm)
        ref = solve(lib, "est_rotation_dev", P, Q, prm)
        assert got[0] == 0
        assert_same(got, ref)


@pytest.mark.parametrize("G,J", [(256, 2048), (1024, 8192)])
def test_noalloc_sampling_rule(lib, G, J):
    """The literal sampling rule through the allocation-free entry point: its
    circle records, partial tiles and padded direction tables (staged in the
    static array's table area) give the same bits as est_rotation_dev, on two
    calls in a row, the second smaller."""
    from paper_2502_06337_amd import SolveParams
    for n, seed in ((20000, 63), (5000, 64)):
        inst = synth.make_instance(n, seed, outlier_rate=0.9)
        P = torch.from_numpy(inst.P).cuda()
        Q = torch.from_numpy(inst.Q).cuda()
        prm = SolveParams(grid=G, angle_bins=360, vote_rule=1, circle_samples=J)
        got = solve(lib, "est_rotation_noalloc_dev", P, Q, prm)
        ref = solve(lib, "est_rotation_dev", P, Q, prm)
        assert got[0] == 0
        assert_same(got, ref)


def test_noalloc_paper_scale(lib):
    """n = 10^6, G = 1024, 64 x 64 refinement, 3600 bins fits the array."""
    from paper_2502_06337_amd import SolveParams
    inst = synth.make_instance(1000000, 2000, outlier_rate=0.9)
    P = torch.from_numpy(inst.P).cuda()
    Q = torch.from_numpy(inst.Q).cuda()
    prm = SolveParams(grid=1024, refine_grid=64, angle_bins=3600)
    got = solve(lib, "est_rotation_noalloc_dev", P, Q, prm)
    ref = solve(lib, "est_rotation_dev", P, Q, prm)
    assert got[0] == 0
    assert_same(got, ref)


def test_noalloc_refuses_what_does_not_fit(lib):
    from paper_2502_06337_amd import SolveParams, ENOMEM, ENODATA
    n = 600000
    P = torch.zeros((3, n), dtype=torch.float32, device="cuda")
    st, res, mask = solve(lib, "est_rotation_noalloc_dev", P, P, SolveParams(grid=4096))
    assert st == ENOMEM
    assert (mask == 7).all()   # nothing ran
    # still usable afterwards, and n < 2 is ENODATA with R = I
    P1 = torch.zeros((3, 1), dtype=torch.float32, device="cuda")
    st, res, mask = solve(lib, "est_rotation_noalloc_dev", P1, P1, SolveParams())
    assert st == ENODATA and mask[0] == 0
    assert np.array_equal(np.asarray(res["R"]), np.eye(3, dtype=np.float32))
