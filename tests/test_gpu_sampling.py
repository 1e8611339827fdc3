"""GPU parity of the literal sampling rule of Algorithm 1 (vote_rule = 1)
against the oracle, through the C ABI.

The coarse accumulator is compared bit for bit with the oracle's sampled grid
(J samples per great circle, one vote per southern sample); full solves with
the oracle's peak search and finishing steps run on that grid (refinement,
angle, inliers by the same rules as the per-cell solve), compared bit for bit;
the least-squares rotation within 2^-22 per entry.
"""
import numpy as np
import pytest

from paper_2502_06337_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LS_TOL = 2.0 ** -22


@pytest.fixture(scope="module")
def aor():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_06337_amd as aor
    aor.load_library()
    return aor


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def gpu_sample_grid(aor, P, Q, G, J):
    prm = aor.SolveParams(grid=G, angle_bins=360, vote_rule=1, circle_samples=J)
    out = aor.solve_debug(dev(P), dev(Q), prm)
    return out["grid"].cpu().numpy().view(np.uint32), out


def assert_result_equal(r, e):
    for key in ("peak_cell", "axis_votes", "fine_cell", "fine_votes", "angle_bin", "angle_votes", "n_inliers",
                "grid"):
        assert r[key] == e[key], (key, r[key], e[key])
    assert np.array_equal(r["axis"].view(np.uint32), e["axis"].view(np.uint32))
    assert np.float32(r["angle"]).view(np.uint32) == np.float32(e["angle"]).view(np.uint32)
    assert np.array_equal(r["R"].view(np.uint32), e["R"].view(np.uint32))


def assert_ls(orc, r, P, Q, mask):
    ref = orc.ls_rotation(P, Q, mask)
    if ref is None:
        assert np.array_equal(r["R_ls"].view(np.uint32), r["R"].view(np.uint32))
    else:
        assert np.max(np.abs(r["R_ls"].astype(np.float64) - ref)) <= LS_TOL


@pytest.mark.parametrize("G,J,n,seed", [
    (64, 100, 700, 1),        # J not a multiple of the wave width: ragged last step
    (128, 1024, 1500, 2),     # the default J = 8 G
    (256, 2048, 1200, 3),
    (64, 20000, 300, 4),      # the whole 64 x 64 grid in one band tile
    (512, 4, 2000, 5),        # four samples per circle
    (512, 37, 1000, 6),       # few samples: every band walks the whole circle
    (2048, 16384, 200, 7),    # band tiles of 16 rows
    (4096, 65536, 40, 8),     # the largest grid and sample count
    (2048, 37, 300, 9),       # whole-circle walks with a row margin above 4095
    (4096, 20, 200, 10),
    (1024, 8192, 600, 11),    # the benchmark's G and J: directions from global memory, runs without an end test
    (256, 8200, 400, 12),     # J not a multiple of 64 there: the last step reads the tables' NaN pads
    (1024, 8046, 400, 13),    # window of 4032 samples: checkpoint intervals of exactly 64, no end test
    (1024, 8044, 400, 14),    # window of 4031: intervals of 63, runs with the end test
])
def test_sample_grid_bit_exact(aor, orc, G, J, n, seed):
    inst = synth.make_instance(n, 5100 + seed)
    g, _ = gpu_sample_grid(aor, inst.P, inst.Q, G, J)
    ref = orc.sample_grid(inst.P, inst.Q, G, J)
    diff = np.argwhere(g != ref)
    assert diff.size == 0, (len(diff), diff[:5])


def test_sample_grid_special_inputs(aor, orc):
    """Equator (every sample on s_z = 0), meridians, huge and tiny
    displacements, zero and non-finite ones (no samples), amid ordinary
    correspondences."""
    rng = np.random.default_rng(52)
    D = rng.uniform(-1, 1, (3, 200)).astype(np.float32)
    D[:, 0] = (0, 0, 1)
    D[:, 1] = (1, 0, 0)
    D[:, 2] = (0, -1, 0)
    D[:, 3] = (0, 0, -3)
    D[:, 4] = (1e-19, 2e-19, 0)      # |d|^2 underflows: no samples
    D[:, 5] = (3e19, 1e19, 2e19)     # |d|^2 overflows: no samples
    D[:, 6] = (1e-10, 0, 1e-10)
    D[:, 7] = (0, 0, 0)
    D[:, 8] = (np.nan, 0, 1)
    D[:, 9] = (np.inf, 1, 0)
    D[:, 10] = (1, 1, 1)
    D[:, 11] = (-1, 1, 1)
    Z = np.zeros_like(D)
    # the equator's samples reach u = 1 exactly (a cell one past the grid
    # before the clamp); the last two also walk runs without an end test
    for G, J in ((64, 512), (128, 1000), (1024, 8192), (256, 8200)):
        g, _ = gpu_sample_grid(aor, Z, D, G, J)
        assert np.array_equal(g, orc.sample_grid(Z, D, G, J))


@pytest.mark.parametrize("seed", [0, 1])
def test_sample_rule_full_solve(aor, orc, seed):
    """C1 shape with the sampling rule, with and without a refinement grid:
    the peak of the sampled grid, then the same finishing steps."""
    inst = synth.make_instance(1000, synth.config_seed(1, seed))
    G, B, J = 256, 360, 2048
    for M in (0, 32):
        prm = aor.SolveParams(grid=G, refine_grid=M, angle_bins=B, vote_rule=1, circle_samples=J)
        out = aor.solve_debug(dev(inst.P), dev(inst.Q), prm)
        grid = orc.sample_grid(inst.P, inst.Q, G, J)
        assert np.array_equal(out["grid"].cpu().numpy().view(np.uint32), grid)
        peak, votes = orc.argmax(grid)
        fin = orc.finish_peak(inst.P, inst.Q, G, M, 1, B, 0.05, peak, votes)
        assert_result_equal(out["result"], fin)
        assert np.array_equal(out["mask"].cpu().numpy(), fin["mask"])
        assert_ls(orc, out["result"], inst.P, inst.Q, fin["mask"])


def test_sample_rule_topk(aor, orc):
    inst = synth.make_instance(3000, 5300, n_rot=3, inlier_frac_each=0.1, sigma=0.01)
    G, B, k, J = 128, 360, 3, 1024
    prm = aor.SolveParams(grid=G, angle_bins=B, nms_radius=5, vote_rule=1, circle_samples=J)
    outs, masks, st = aor.est_rotations_topk(dev(inst.P), dev(inst.Q), k, prm)
    masks = masks.cpu().numpy()
    grid = orc.sample_grid(inst.P, inst.Q, G, J)
    peaks = orc.topk_peaks(grid, k, 5)
    assert len(outs) == len(peaks) == 3
    for t, (pk, votes) in enumerate(peaks):
        fin = orc.finish_peak(inst.P, inst.Q, G, 0, 1, B, 0.05, pk, votes)
        assert_result_equal(outs[t], fin)
        assert np.array_equal(masks[t], fin["mask"])


def test_batch_mixes_rules(aor):
    """Instances with either rule in one batched call: each result equals its
    one-at-a-time solve."""
    sizes = [1200, 800, 0, 1500]
    insts = [synth.make_instance(max(n, 1), 5400 + t) for t, n in enumerate(sizes)]
    P = np.concatenate([i.P[:, :n] for i, n in zip(insts, sizes)], axis=1)
    Q = np.concatenate([i.Q[:, :n] for i, n in zip(insts, sizes)], axis=1)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    opts = [(1, 512), (0, 0), (1, 0), (1, 20000)]
    prms = [aor.SolveParams(grid=128, angle_bins=360, vote_rule=r, circle_samples=j) for r, j in opts]
    outs, mask, st = aor.est_rotation_batch(dev(P), dev(Q), off, prms)
    mask = mask.cpu().numpy()
    for t, n in enumerate(sizes):
        if n < 2:
            continue
        r1, m1, _ = aor.est_rotation(insts[t].P[:, :n], insts[t].Q[:, :n], prms[t])
        assert_result_equal(outs[t], r1)
        assert np.array_equal(outs[t]["R_ls"].view(np.uint32), r1["R_ls"].view(np.uint32))
        assert np.array_equal(mask[off[t]:off[t + 1]], m1)


def test_sample_rule_at_full_grid_and_samples(aor, orc):
    """The benchmark's grid and default sample count (G = 1024, J = 8192) on
    3e4 correspondences of its input distribution: the grid bit for bit."""
    inst = synth.make_instance(30_000, 2000)
    g, out = gpu_sample_grid(aor, inst.P, inst.Q, 1024, 0)
    ref = orc.sample_grid(inst.P, inst.Q, 1024, 8192)
    assert np.array_equal(g, ref)
    assert out["result"]["peak_cell"] == int(np.argmax(ref.ravel()))


@pytest.mark.parametrize("d", [(0.3, -0.2, 0.9), (0.0, 0.0, 1.0)])
def test_sample_counts_in_packed_tiles(aor, orc, d):
    """2.1e5 copies of one circle (items of 6544 circles, the most the 16-bit
    band counters allow at J = 8 G): every cell equals the copy count times the
    oracle's count for one circle."""
    n, G, J = 210_000, 128, 1024
    Q = np.tile(np.asarray(d, np.float32)[:, None], (1, n))
    P = np.zeros_like(Q)
    g, _ = gpu_sample_grid(aor, P, Q, G, J)
    one = orc.sample_grid(P[:, :1], Q[:, :1], G, J).astype(np.int64)
    assert np.array_equal(g.astype(np.int64), one * n)


def test_graph_replays_with_rules_and_angle_options(aor):
    """Captured batch graphs with the sampling rule and the angle options,
    replayed with the same and with changed compositions, eager solves and
    synchronisations in between: every launch equals the one-at-a-time
    results."""
    comps = [[1500, 900, 2500], [1500, 900, 2500], [700, 3000, 1200, 400], [1500, 900, 2500]]
    for rep, sizes in enumerate(comps):
        insts = [synth.make_instance(n, 5600 + 13 * t, outlier_rate=0.85) for t, n in enumerate(sizes)]
        P = np.concatenate([i.P for i in insts], axis=1)
        Q = np.concatenate([i.Q for i in insts], axis=1)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
        prms = [aor.SolveParams(grid=128, angle_bins=360, vote_rule=(t + rep) % 2, circle_samples=512,
                                angle_gate=t % 2, angle_refine=(4 if t % 3 else 0)) for t in range(len(sizes))]
        outs, mask, _ = aor.est_rotation_batch(dev(P), dev(Q), off, prms)
        mask = mask.cpu().numpy()
        torch.cuda.synchronize()
        for t in range(len(sizes)):
            r1, m1, _ = aor.est_rotation(insts[t].P, insts[t].Q, prms[t])
            assert_result_equal(outs[t], r1)
            assert outs[t]["angle_fine_bin"] == r1["angle_fine_bin"]
            assert np.array_equal(mask[off[t]:off[t + 1]], m1), (rep, t)


def test_sample_rule_full_size_additivity(aor):
    """The benchmark's launch (n = 1e6, G = 1024, J = 8192): the grid of all
    circles equals the sum of the grids of two unequal parts, whose chunks,
    band items and partial arenas differ from the full launch's, and every
    circle casts about J/2 votes."""
    inst = synth.make_instance(1_000_000, 2000)
    g_all, _ = gpu_sample_grid(aor, inst.P, inst.Q, 1024, 0)
    k = 377_777
    g_a, _ = gpu_sample_grid(aor, inst.P[:, :k], inst.Q[:, :k], 1024, 0)
    g_b, _ = gpu_sample_grid(aor, inst.P[:, k:], inst.Q[:, k:], 1024, 0)
    assert np.array_equal(g_all.astype(np.int64), g_a.astype(np.int64) + g_b.astype(np.int64))
    total = int(g_all.astype(np.int64).sum())
    assert abs(total - 4096 * 1_000_000) <= 1_000_000
