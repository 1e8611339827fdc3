"""Autotuner of the coarse vote's work split: a tuned plan changes speed,
never results, and the tuning table survives a save/load round trip."""
import os

import numpy as np
import pytest

from paper_2502_06337_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def aor():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_06337_amd as aor
    aor.load_library()
    return aor


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_tuned_solve_is_bit_identical(aor, tmp_path):
    inst = synth.make_instance(60000, 4242, outlier_rate=0.9)
    P, Q = dev(inst.P), dev(inst.Q)
    prm = aor.SolveParams(grid=512, refine_grid=32, angle_bins=720)
    aor.tuner_clear()
    r0, m0, s0 = aor.est_rotation(P, Q, prm)
    g0 = aor.coarse_grid(P, Q, 512).cpu().numpy()
    chosen = aor.autotune(P, Q, prm)
    assert chosen["grid"] == 512 and chosen["vote_ms"] > 0
    assert chosen["tile_cells"] in (16384, 32768, 65536)
    assert aor.tuner_get(512, 60000) == chosen
    r1, m1, s1 = aor.est_rotation(P, Q, prm)
    g1 = aor.coarse_grid(P, Q, 512).cpu().numpy()
    assert s0 == s1
    assert np.array_equal(g0, g1)
    for k in ("peak_cell", "axis_votes", "fine_cell", "fine_votes", "angle_bin", "angle_votes", "n_inliers"):
        assert r0[k] == r1[k], k
    assert np.array_equal(r0["R"].view(np.uint32), r1["R"].view(np.uint32))
    assert torch.equal(m0, m1)
    # every candidate split, forced through the table, gives the same grid
    path = os.path.join(str(tmp_path), "tune.jsonl")
    aor.tuner_save(path)
    text = open(path).read()
    assert '"grid": 512' in text
    for tile in (16384, 32768, 65536):
        for target in (7.5e5, 6e6):
            line = text.splitlines()[0]
            import json
            d = json.loads(line)
            d["tile_cells"], d["vote_target"] = tile, target
            with open(path, "w") as f:
                f.write(json.dumps(d) + "\n")
            aor.tuner_clear()
            aor.tuner_load(path)
            assert aor.tuner_get(512, 60000)["tile_cells"] == tile
            g = aor.coarse_grid(P, Q, 512).cpu().numpy()
            assert np.array_equal(g, g0), (tile, target)
    aor.tuner_clear()
