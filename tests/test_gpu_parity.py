"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Vote grids, fine grids and histograms must match bit for bit; peak indices,
angle bins and inlier masks exactly; the axis, angle and R are compared bit
for bit as well (both sides evaluate the same binary32 expressions), which
is stricter than the 1e-4 rad tolerance the method asks for.
"""
import math

import numpy as np
import pytest

from paper_2502_06337_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def aor():
    _need_gpu()
    import paper_2502_06337_amd as aor
    aor.load_library()
    return aor


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def gpu_grid(aor, P, Q, G):
    g = aor.coarse_grid(dev(P), dev(Q), G)
    torch.cuda.synchronize()
    return g.cpu().numpy().view(np.uint32)


def assert_result_equal(r_gpu, r_or, check_mask=True):
    for key in ("peak_cell", "axis_votes", "fine_cell", "fine_votes", "angle_bin", "angle_votes", "n_inliers",
                "grid"):
        assert r_gpu[key] == r_or[key], (key, r_gpu[key], r_or[key])
    assert np.array_equal(r_gpu["axis"].view(np.uint32), r_or["axis"].view(np.uint32)), (r_gpu["axis"], r_or["axis"])
    assert np.float32(r_gpu["angle"]).view(np.uint32) == np.float32(r_or["angle"]).view(np.uint32)
    assert np.array_equal(r_gpu["R"].view(np.uint32), r_or["R"].view(np.uint32)), (r_gpu["R"], r_or["R"])
    if "R_ls" in r_gpu and "R_ls" in r_or:   # two GPU results: the least-squares rotation too, bit for bit
        assert np.array_equal(r_gpu["R_ls"].view(np.uint32), r_or["R_ls"].view(np.uint32))


# The least-squares rotation on the inlier set is accumulated in float64 in a
# different order than the oracle's matrix product and solved by a different
# method (quaternion eigenvector vs SVD); both are float64-accurate to about
# 1e-14 on these well-conditioned sets, and the GPU rounds its rotation once to
# binary32, so entries agree within one binary32 step at 1.0 (2^-23), tested
# with a margin of two.
LS_TOL = 2.0 ** -22


def assert_ls(orc, r_gpu, P, Q, mask):
    ref = orc.ls_rotation(P, Q, mask)
    if ref is None:
        assert np.array_equal(r_gpu["R_ls"].view(np.uint32), r_gpu["R"].view(np.uint32))
        return
    err = np.max(np.abs(r_gpu["R_ls"].astype(np.float64) - ref))
    assert err <= LS_TOL, err


# ------------------------------------------------------------- coarse grid
@pytest.mark.parametrize("G", [64, 128, 256])
@pytest.mark.parametrize("seed", [0, 1])
def test_coarse_grid_bit_exact(aor, orc, G, seed):
    inst = synth.make_instance(700, 3000 + seed)
    g_gpu = gpu_grid(aor, inst.P, inst.Q, G)
    g_or = orc.coarse_grid(inst.P, inst.Q, G)
    diff = np.argwhere(g_gpu != g_or)
    assert diff.size == 0, (len(diff), diff[:10], g_gpu[tuple(diff[0])], g_or[tuple(diff[0])])


@pytest.mark.parametrize("G", [512, 2048, 4096])
def test_coarse_grid_bit_exact_large_grids(aor, orc, G):
    """Band widths of 128, 32 and 16 lines (16-bit tiles of 65536 cells); fewer
    correspondences on the finer grids keep the oracle's full grid quick."""
    inst = synth.make_instance(1500 if G <= 512 else 200, 3100 + G)
    g_gpu = gpu_grid(aor, inst.P, inst.Q, G)
    g_or = orc.coarse_grid(inst.P, inst.Q, G)
    diff = np.argwhere(g_gpu != g_or)
    assert diff.size == 0, (len(diff), diff[:10])


def test_coarse_grid_counts_beyond_16_bits(aor, orc):
    """70000 copies of one correspondence at G = 1024: every cell on its curve
    collects 70000 votes, 64512 of them from one work item; the 16-bit band
    counters must neither overflow nor carry into the neighbouring line."""
    G, n = 1024, 70000
    one = synth.make_instance(1, 77)
    P = np.repeat(one.P, n, axis=1)
    Q = np.repeat(one.Q, n, axis=1)
    g_gpu = gpu_grid(aor, P, Q, G)
    g_one = orc.coarse_grid(one.P, one.Q, G).astype(np.uint64)
    assert g_one.sum() > 0
    assert np.array_equal(g_gpu.astype(np.uint64), g_one * n)


def special_cases():
    """Lines, the unit circle, axis-aligned and near-degenerate displacements."""
    rows = []
    vals = [(0.0, 0.0, 0.5), (0.75, 0.0, 0.0), (0.0, 0.3, 0.0), (0.5, 0.5, 0.0), (0.5, -0.5, 0.0),
            (1e-3, 1.0, 1e-7), (1.0, 1e-3, 1e-7), (0.3, 0.4, 1e-30), (1e-20, 0.0, 1.0), (0.0, 1e-20, 1.0),
            (0.6, 0.8, 0.0), (0.70710677, 0.70710677, 1e-3), (1e-35, 2e-35, 3e-35), (1e-36, 0.0, 0.0),
            (3e37, 1e37, 2e37), (0.0, 0.0, 0.0), (np.inf, 0.0, 0.0), (np.nan, 1.0, 1.0),
            (0.2, 0.1, -0.3), (-0.9, 0.01, -0.001), (2.0, -3.0, 0.5)]
    for d in vals:
        rows.append(d)
    D = np.array(rows, dtype=np.float32).T
    Q = np.zeros_like(D)
    return D, Q


@pytest.mark.parametrize("G", [64, 256, 1024])
def test_coarse_grid_special_cases(aor, orc, G):
    P, Q = special_cases()
    for i in range(P.shape[1]):
        g_gpu = gpu_grid(aor, P[:, i:i + 1], Q[:, i:i + 1], G)
        g_or = orc.coarse_grid(P[:, i:i + 1], Q[:, i:i + 1], G)
        assert np.array_equal(g_gpu, g_or), (i, P[:, i], int((g_gpu != g_or).sum()))


def test_coarse_grid_ragged_and_empty(aor, orc):
    G = 128
    for n in (1, 2, 3, 1023, 1025, 4097):
        inst = synth.make_instance(n, 40 + n, outlier_rate=0.5)
        g_gpu = gpu_grid(aor, inst.P, inst.Q, G)
        g_or = orc.coarse_grid(inst.P, inst.Q, G)
        assert np.array_equal(g_gpu, g_or), n
    z = np.zeros((3, 0), dtype=np.float32)
    g = aor.coarse_grid(torch.zeros((3, 0), device="cuda"), torch.zeros((3, 0), device="cuda"), G)
    assert int(g.sum()) == 0


# ------------------------------------------------------------- full solves
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_solve_c1_shape(aor, orc, seed):
    """n = 1000, 90% outliers, G = 256, B = 360, no refinement."""
    inst = synth.make_instance(1000, synth.config_seed(1, seed))
    prm = aor.SolveParams(grid=256, angle_bins=360)
    out = aor.solve_debug(dev(inst.P), dev(inst.Q), prm)
    r_or = orc.solve(inst.P, inst.Q, G=256, B=360, want_grids=True)
    assert np.array_equal(out["grid"].cpu().numpy().view(np.uint32), r_or["grid_full"])
    assert np.array_equal(out["hist"].cpu().numpy().view(np.uint32), r_or["hist"])
    assert_result_equal(out["result"], r_or)
    assert np.array_equal(out["mask"].cpu().numpy(), r_or["mask"])
    assert_ls(orc, out["result"], inst.P, inst.Q, r_or["mask"])


@pytest.mark.parametrize("seed", [0, 1])
def test_solve_with_refinement(aor, orc, seed):
    inst = synth.make_instance(1500, 77 + seed)
    G, M, B = 256, 64, 3600
    prm = aor.SolveParams(grid=G, refine_grid=M, angle_bins=B)
    out = aor.solve_debug(dev(inst.P), dev(inst.Q), prm)
    r_or = orc.solve(inst.P, inst.Q, G=G, B=B, M=M, want_grids=True)
    assert np.array_equal(out["grid"].cpu().numpy().view(np.uint32), r_or["grid_full"])
    assert np.array_equal(out["fine"].cpu().numpy().view(np.uint32), r_or["fine"])
    assert np.array_equal(out["hist"].cpu().numpy().view(np.uint32), r_or["hist"])
    assert_result_equal(out["result"], r_or)
    assert_ls(orc, out["result"], inst.P, inst.Q, r_or["mask"])


def test_host_entry_point_matches_device(aor, orc):
    inst = synth.make_instance(1200, 5)
    prm = aor.SolveParams(grid=128, angle_bins=360)
    r_h, m_h, st_h = aor.est_rotation(inst.P, inst.Q, prm)
    r_d, m_d, st_d = aor.est_rotation(dev(inst.P), dev(inst.Q), prm)
    assert st_h == st_d == 0
    assert_result_equal(r_h, r_d)
    assert np.array_equal(m_h, m_d.cpu().numpy())
    r_or = orc.solve(inst.P, inst.Q, G=128, B=360)
    assert_result_equal(r_h, r_or)


def test_topk_parity(aor, orc):
    inst = synth.make_instance(1500, 99, n_rot=3, inlier_frac_each=0.1, sigma=0.01)
    G, B, k = 128, 360, 3
    prm = aor.SolveParams(grid=G, angle_bins=B, nms_radius=5)
    outs, masks, st = aor.est_rotations_topk(inst.P, inst.Q, k, prm)
    ors = orc.solve_topk(inst.P, inst.Q, G=G, B=B, k=k, rad=5)
    assert len(outs) == len(ors)
    for t, (a, b) in enumerate(zip(outs, ors)):
        assert_result_equal(a, b)
        assert np.array_equal(masks[t], b["mask"])
        assert_ls(orc, a, inst.P, inst.Q, b["mask"])


def test_topk_with_refinement_parity(aor, orc):
    """Multi-rotation shape (three rotations, 10% inliers each, 70% outliers)
    with a refinement grid per peak and suppression of radius 5."""
    inst = synth.make_instance(3000, 303, n_rot=3, inlier_frac_each=0.1, sigma=0.01)
    G, B, k, M = 128, 720, 3, 16
    prm = aor.SolveParams(grid=G, angle_bins=B, nms_radius=5, refine_grid=M)
    outs, masks, st = aor.est_rotations_topk(dev(inst.P), dev(inst.Q), k, prm)
    masks = masks.cpu().numpy()
    ors = orc.solve_topk(inst.P, inst.Q, G=G, B=B, k=k, rad=5, M=M)
    assert len(outs) == len(ors) == 3
    for t, (a, b) in enumerate(zip(outs, ors)):
        assert_result_equal(a, b)
        assert np.array_equal(masks[t], b["mask"])


@pytest.mark.parametrize("G,n,target", [(512, 12000, 2e4), (1024, 4000, 1e4), (2048, 2500, 1e4)])
def test_many_items_per_band_whole_grid(aor, orc, tmp_path, G, n, target):
    """The coarse vote with a small votes-per-item target forced through the
    tuner table, so that every band of every pass is split over several work
    items that flush into the same cells, on varied curves (90% outliers):
    the whole grid equals the oracle's, bit for bit, and equals the grid of
    the default split."""
    import json
    import _oracle_par
    inst = synth.make_instance(n, 7000 + G, outlier_rate=0.9)
    P, Q = dev(inst.P), dev(inst.Q)
    prm = aor.SolveParams(grid=G, angle_bins=360)
    aor.tuner_clear()
    g_default = gpu_grid(aor, inst.P, inst.Q, G).ravel()
    aor.autotune(P, Q, prm)
    path = str(tmp_path / "split.jsonl")
    aor.tuner_save(path)
    d = json.loads(open(path).read().splitlines()[0])
    d["tile_cells"], d["vote_target"] = 65536, target
    with open(path, "w") as f:
        f.write(json.dumps(d) + "\n")
    aor.tuner_clear()
    aor.tuner_load(path)
    assert aor.tuner_get(G, n)["vote_target"] == pytest.approx(target)
    g_split = gpu_grid(aor, inst.P, inst.Q, G).ravel()
    aor.tuner_clear()
    ref = _oracle_par.coarse_grid(orc, inst.P, inst.Q, G).ravel()
    assert np.array_equal(g_split, ref), np.flatnonzero(g_split != ref)[:20]
    assert np.array_equal(g_default, ref)


def _broad_and_rim_instance(G, n=20000, seed=77):
    """Three rotations: a strong one with noisy inliers (sigma = 0.04) whose
    peak spreads past 5 cells at G = 128, and two weaker ones, one with its axis
    2.5 cells from the disk rim (the oracle's pins use the same shape)."""
    rng = np.random.default_rng(seed)
    P = rng.uniform(-1, 1, (3, n))
    Q = rng.uniform(-1, 1, (3, n))
    h = 2.0 / G
    spec = [((0.05, -0.1), 1.0, 0.4), ((-0.45, 0.35), -2.0, 0.12), ((1 - 2.5 * h, 0.02), 2.4, 0.12)]
    perm = rng.permutation(n)
    st = 0
    for (u, v), t, frac in spec:
        s = u * u + v * v
        a = np.array([2 * u, 2 * v, s - 1]) / (1 + s)
        K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
        R = np.eye(3) + math.sin(t) * K + (1 - math.cos(t)) * (K @ K)
        cnt = int(frac * n)
        idx = perm[st:st + cnt]
        st += cnt
        Q[:, idx] = R @ P[:, idx] + 0.04 * rng.standard_normal((3, cnt))
    return P.astype(np.float32), Q.astype(np.float32)


def test_topk_local_maxima_rim_axis(aor, orc):
    """Sec. IV-D: a broad peak's flank outvotes a rim axis's peak; the peaks
    are local maxima within the radius, so the rim axis is the third."""
    G, B, k = 128, 360, 4
    P, Q = _broad_and_rim_instance(G)
    prm = aor.SolveParams(grid=G, angle_bins=B, nms_radius=5)
    outs, masks, st = aor.est_rotations_topk(dev(P), dev(Q), k, prm)
    masks = masks.cpu().numpy()
    ors = orc.solve_topk(P, Q, G=G, B=B, k=k, rad=5)
    assert len(outs) == len(ors) >= 3
    for t, (a, b) in enumerate(zip(outs, ors)):
        assert_result_equal(a, b)
        assert np.array_equal(masks[t], b["mask"])


@pytest.mark.parametrize("rad", [1, 3, 12, 32, 40])
def test_topk_radius_parity(aor, orc, rad):
    """Local maxima within radii of 1 to 40 cells (disk rows clipped at the
    grid edge, ties between equal counts at small n; radii above 32 take the
    kernel's path without LDS staging), up to 6 peaks."""
    inst = synth.make_instance(2500, 400 + rad, n_rot=3, inlier_frac_each=0.1, sigma=0.02)
    G, B, k = 64 if rad in (12, 32) else 128, 360, 6
    prm = aor.SolveParams(grid=G, angle_bins=B, nms_radius=rad)
    outs, masks, st = aor.est_rotations_topk(dev(inst.P), dev(inst.Q), k, prm)
    masks = masks.cpu().numpy()
    ors = orc.solve_topk(inst.P, inst.Q, G=G, B=B, k=k, rad=rad)
    assert len(outs) == len(ors)
    for t, (a, b) in enumerate(zip(outs, ors)):
        assert_result_equal(a, b)
        assert np.array_equal(masks[t], b["mask"])


def test_enodata(aor):
    P = np.zeros((3, 1), dtype=np.float32)
    r, m, st = aor.est_rotation(P, P, aor.SolveParams(grid=64))
    assert st == aor.ENODATA
    assert np.array_equal(r["R"], np.eye(3, dtype=np.float32))
    assert np.array_equal(r["R_ls"], np.eye(3, dtype=np.float32))
    P = np.ones((3, 10), dtype=np.float32)
    r, m, st = aor.est_rotation(P, P, aor.SolveParams(grid=64))
    assert st == aor.ENODATA
    assert np.array_equal(r["R"], np.eye(3, dtype=np.float32))
    assert np.array_equal(r["R_ls"], np.eye(3, dtype=np.float32))


# ------------------------------------------------------------------ batching
def test_batch_matches_single_solves(aor, orc):
    """Instances of uneven size in one batched call: each result is
    bit-identical to the one-at-a-time solve, and to the oracle."""
    sizes = [1500, 0, 700, 1, 3000, 2, 900, 4100]
    insts = [synth.make_instance(n, 500 + t, outlier_rate=0.8) for t, n in enumerate(sizes)]
    P = np.concatenate([i.P for i in insts], axis=1)
    Q = np.concatenate([i.Q for i in insts], axis=1)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    prms = [aor.SolveParams(grid=(128 if t % 2 else 0), angle_bins=360, refine_grid=(16 if t % 3 == 0 else 0))
            for t in range(len(sizes))]
    outs, mask, st = aor.est_rotation_batch(P, Q, off, prms)
    outs_d, mask_d, st_d = aor.est_rotation_batch(dev(P), dev(Q), off, prms)
    assert np.array_equal(mask, mask_d.cpu().numpy())
    for t, n in enumerate(sizes):
        assert_result_equal(outs[t], outs_d[t])
        if n < 2:
            assert np.array_equal(outs[t]["R"], np.eye(3, dtype=np.float32))
            continue
        r1, m1, _ = aor.est_rotation(insts[t].P, insts[t].Q, prms[t])
        assert_result_equal(outs[t], r1)
        assert np.array_equal(mask[off[t]:off[t + 1]], m1)
        G = prms[t].grid or aor.grid_for_n(n)
        r_or = orc.solve(insts[t].P, insts[t].Q, G=G, B=360, M=prms[t].refine_grid)
        assert_result_equal(outs[t], r_or)
        assert_ls(orc, outs[t], insts[t].P, insts[t].Q, r_or["mask"])


def test_batch_graph_relaunched_with_changing_batches(aor):
    """Batches run as one captured graph that is updated in place or rebuilt
    from call to call.  Several batches of different composition, with eager
    single solves and synchronisations in between, must each equal the
    one-at-a-time results."""
    rng = np.random.default_rng(7)
    for rep in range(4):
        nb = [3, 5, 3, 8][rep]
        sizes = [int(x) for x in rng.integers(300, 5000, nb)]
        insts = [synth.make_instance(n, 7000 + 37 * rep + t, outlier_rate=0.85) for t, n in enumerate(sizes)]
        P = np.concatenate([i.P for i in insts], axis=1)
        Q = np.concatenate([i.Q for i in insts], axis=1)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
        prm = aor.SolveParams(angle_bins=360, refine_grid=(16 if rep % 2 else 0))
        outs, mask, _ = aor.est_rotation_batch(dev(P), dev(Q), off, prm)
        mask = mask.cpu().numpy()
        torch.cuda.synchronize()
        for t in range(nb):
            r1, m1, _ = aor.est_rotation(insts[t].P, insts[t].Q, prm)
            assert_result_equal(outs[t], r1)
            assert np.array_equal(mask[off[t]:off[t + 1]], m1), (rep, t)


def test_batch_graph_replayed_on_new_data(aor):
    """A batched call with the same layout as the previous one (offsets,
    parameters, device pointers) launches the recorded graph again: with the
    inputs overwritten in place between calls, and with a single solve in
    between (which forces a new recording), every result equals the
    one-at-a-time solve of the current data."""
    sizes = [2000, 500, 3000, 64]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    prm = aor.SolveParams(angle_bins=360, refine_grid=16)
    Pd = torch.zeros((3, int(off[-1])), dtype=torch.float32, device="cuda")
    Qd = torch.zeros_like(Pd)
    for rep, single_between in enumerate([False, False, True, False, False]):
        insts = [synth.make_instance(n, 8100 + 10 * rep + t, outlier_rate=0.85) for t, n in enumerate(sizes)]
        Pd.copy_(torch.from_numpy(np.concatenate([i.P for i in insts], axis=1)))
        Qd.copy_(torch.from_numpy(np.concatenate([i.Q for i in insts], axis=1)))
        if single_between:
            aor.est_rotation(insts[0].P, insts[0].Q, prm)
        outs, _, _ = aor.est_rotation_batch(Pd, Qd, off, prm, want_mask=False)
        torch.cuda.synchronize()
        for t in range(len(sizes)):
            r1, _, _ = aor.est_rotation(insts[t].P, insts[t].Q, prm)
            assert_result_equal(outs[t], r1)
        # the solo solves above used the workspace: the next call records again,
        # and the one after it replays
        outs2, _, _ = aor.est_rotation_batch(Pd, Qd, off, prm, want_mask=False)
        outs3, _, _ = aor.est_rotation_batch(Pd, Qd, off, prm, want_mask=False)
        torch.cuda.synchronize()
        for t in range(len(sizes)):
            assert_result_equal(outs2[t], outs[t])
            assert_result_equal(outs3[t], outs[t])


def test_determinism_repeat_and_permutation(aor):
    """Repeated solves give identical bits, and a permutation of the
    correspondences gives the identical accumulator, result and (permuted)
    mask: every count is an integer sum and every float a fixed expression,
    whatever the work split and the order in which work-groups run."""
    inst = synth.make_instance(200000, 4321, outlier_rate=0.9)
    prm = aor.SolveParams(grid=1024, refine_grid=64, angle_bins=3600)
    P, Q = dev(inst.P), dev(inst.Q)
    base = aor.solve_debug(P, Q, prm)
    for _ in range(3):
        again = aor.solve_debug(P, Q, prm)
        assert torch.equal(again["grid"], base["grid"]) and torch.equal(again["fine"], base["fine"])
        assert torch.equal(again["hist"], base["hist"]) and torch.equal(again["mask"], base["mask"])
        assert_result_equal(again["result"], base["result"])
        assert np.array_equal(np.asarray(again["result"]["R_ls"]).view(np.uint32),
                              np.asarray(base["result"]["R_ls"]).view(np.uint32))
    perm = np.random.default_rng(5).permutation(inst.n)
    Pp, Qp = dev(inst.P[:, perm]), dev(inst.Q[:, perm])
    other = aor.solve_debug(Pp, Qp, prm)
    assert torch.equal(other["grid"], base["grid"]) and torch.equal(other["fine"], base["fine"])
    assert torch.equal(other["hist"], base["hist"])
    assert_result_equal(other["result"], base["result"])
    assert np.array_equal(other["mask"].cpu().numpy(), base["mask"].cpu().numpy()[perm])


# ------------------------------------------------------ full size, sampled
def test_paper_scale_sampled_parity(aor, orc):
    """n = 1e6, G = 1024 + 64x64 refinement, B = 3600 (the benchmark's launch
    configuration): sampled coarse and fine cells recomputed by the oracle one
    by one, the full histogram, axis, R and mask against the oracle."""
    n, G, M, B = 1_000_000, 1024, 64, 3600
    inst = synth.make_instance(n, 2000)
    prm = aor.SolveParams(grid=G, refine_grid=M, angle_bins=B)
    out = aor.solve_debug(dev(inst.P), dev(inst.Q), prm)
    r = out["result"]
    grid = out["grid"].cpu().numpy().view(np.uint32)
    # the peak is the argmax of the returned grid (ties to the lowest index)
    assert r["peak_cell"] == int(np.argmax(grid.ravel())) and r["axis_votes"] == int(grid.max())
    rng = np.random.default_rng(7)
    ix, iy = r["peak_cell"] % G, r["peak_cell"] // G
    cells = [(ix + dx, iy + dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1)]
    cells += [tuple(int(v) for v in rng.integers(0, G, 2)) for _ in range(12)]
    for (cx, cy) in cells:
        assert grid[cy, cx] == orc.coarse_cell(inst.P, inst.Q, G, cx, cy), (cx, cy)
    win = orc.fine_window(G, M, 1, ix, iy)
    fine = out["fine"].cpu().numpy().view(np.uint32)
    fc = r["fine_cell"]
    assert fc == int(np.argmax(fine.ravel()))
    for (jx, jy) in [(fc % M, fc // M)] + [tuple(int(v) for v in rng.integers(0, M, 2)) for _ in range(6)]:
        assert fine[jy, jx] == orc.fine_cell(inst.P, inst.Q, win, jx, jy), (jx, jy)
    fin = orc.finish_peak(inst.P, inst.Q, G, M, 1, B, 0.05, r["peak_cell"], r["axis_votes"], want_grids=True)
    assert np.array_equal(out["hist"].cpu().numpy().view(np.uint32), fin["hist"])
    assert_result_equal(r, fin)
    assert np.array_equal(out["mask"].cpu().numpy(), fin["mask"])
    assert orc.rotation_error_deg(inst.R_gt[0], r["R"]) < 0.5
    assert_ls(orc, r, inst.P, inst.Q, fin["mask"])
    # the least-squares rotation on 1e5 inliers with sigma = 0.01 lands far below a cell
    assert orc.rotation_error_deg(inst.R_gt[0], r["R_ls"]) < 0.01
    # the same launch with coarse-to-fine angle voting (gate on the 3 x 3
    # window, 36000 fine bins): the axis stage is unchanged, the angle stage
    # against the oracle's coarse-to-fine vote on the oracle's axis
    prm = aor.SolveParams(grid=G, refine_grid=M, angle_bins=B, angle_gate=1, angle_refine=10)
    r2, m2, st = aor.est_rotation(dev(inst.P), dev(inst.Q), prm)
    c2f = orc.angle_coarse_to_fine(inst.P, inst.Q, fin["axis"], G, fin["peak_cell"], 1, B, 10)
    mask2, cnt2 = orc.inliers(c2f["R"], inst.P, inst.Q, 0.05)
    for key in ("peak_cell", "fine_cell", "axis_votes", "fine_votes"):
        assert r2[key] == r[key]
    for key in ("angle_bin", "angle_votes", "angle_fine_bin", "angle_fine_votes"):
        assert r2[key] == c2f[key], (key, r2[key], c2f[key])
    assert np.float32(r2["angle"]).view(np.uint32) == np.float32(c2f["angle"]).view(np.uint32)
    assert np.array_equal(r2["R"].view(np.uint32), np.asarray(c2f["R"], np.float32).view(np.uint32))
    assert r2["n_inliers"] == cnt2
    assert np.array_equal(m2.cpu().numpy(), mask2)
    assert_ls(orc, r2, inst.P, inst.Q, mask2)


def rot(axis, t):
    axis = np.asarray(axis, dtype=np.float64) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(t) * K + (1 - math.cos(t)) * K @ K


@pytest.mark.parametrize("uv", [(0.995, 0.01), (-0.02, -0.997), (0.70, 0.70)])
def test_refinement_window_at_grid_edge(aor, orc, uv):
    """Axis projecting next to the border of the grid: the refinement window
    is clipped to 2 x 3 (or 2 x 2) coarse cells, so its fine cells are not
    square."""
    u, v = uv
    s = u * u + v * v
    r = np.array([2 * u / (1 + s), 2 * v / (1 + s), (s - 1) / (1 + s)])
    rng = np.random.default_rng(int(1000 * (u + 2)))
    n = 1200
    P = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    Q = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    Q[:, :300] = (rot(r, 0.7) @ P[:, :300].astype(np.float64)).astype(np.float32)
    G, M, B = 128, 32, 720
    prm = aor.SolveParams(grid=G, refine_grid=M, angle_bins=B)
    out = aor.solve_debug(dev(P), dev(Q), prm)
    r_or = orc.solve(P, Q, G=G, B=B, M=M, want_grids=True)
    assert np.array_equal(out["grid"].cpu().numpy().view(np.uint32), r_or["grid_full"])
    assert np.array_equal(out["fine"].cpu().numpy().view(np.uint32), r_or["fine"])
    assert_result_equal(out["result"], r_or)
