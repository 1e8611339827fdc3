"""Request loop: continuous batching on the GPU.

Requests of mixed size submitted from several threads at staggered times
are admitted while others run; each result must be bit-identical to the
same problem solved alone with est_rotation and to the CPU oracle's solve.
"""
import threading
import time

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


def same(a, b):
    for k in ("peak_cell", "axis_votes", "fine_cell", "angle_bin", "angle_votes", "n_inliers", "grid"):
        if a[k] != b[k]:
            return False
    return np.array_equal(a["R"].view(np.uint32), b["R"].view(np.uint32))


def matches_oracle(r, o):
    for k in ("peak_cell", "axis_votes", "fine_cell", "fine_votes", "angle_bin", "angle_votes", "n_inliers",
              "grid"):
        if int(r[k]) != int(o[k]):
            return False
    return (np.array_equal(np.asarray(r["axis"], np.float32).view(np.uint32), o["axis"].view(np.uint32))
            and np.array_equal(r["R"].view(np.uint32), o["R"].view(np.uint32)))


def oracle_solutions(orc, aor, probs, G=None, B=360, M=16):
    """The oracle's solve of every problem (threads: the oracle's C code runs
    without the interpreter lock), with the grid the library picks for n."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    def one(p):
        if p.n < 2:
            return None
        return orc.solve(p.P, p.Q, G=G or aor.grid_for_n(p.n), B=B, M=M)
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, probs))


def test_served_results_equal_solo(aor, orc):
    rng = np.random.default_rng(3)
    sizes = [int(x) for x in np.exp(rng.uniform(np.log(300), np.log(30000), 40))] + [0, 1, 5]
    probs = [synth.make_instance(n, 9000 + t, outlier_rate=0.85) for t, n in enumerate(sizes)]
    prm = aor.SolveParams(angle_bins=360, refine_grid=16)
    srv = aor.Server(hbm_budget_bytes=64 << 20, max_slots=8)
    ids = [None] * len(probs)

    def client(lo, hi):
        for t in range(lo, hi):
            ids[t] = srv.submit(probs[t].P, probs[t].Q, prm)
            time.sleep(0.001 * (t % 3))

    th = [threading.Thread(target=client, args=(k, min(k + 11, len(probs)))) for k in range(0, len(probs), 11)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    served = []
    for t, rid in enumerate(ids):
        st, res, mask = srv.poll(rid, timeout_us=-1)
        served.append((st, res, mask))
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == len(probs)
    assert 0 < stats["p50_us"] <= stats["p99_us"]
    for t, p in enumerate(probs):
        st, res, mask = served[t]
        if p.n < 2:
            assert st == aor.ENODATA
            continue
        r1, m1, st1 = aor.est_rotation(p.P, p.Q, prm)
        assert st == st1
        assert same(res, r1), t
        assert np.array_equal(mask, m1)
    # and every served result is the oracle's, bit for bit
    refs = oracle_solutions(orc, aor, probs)
    for t, p in enumerate(probs):
        if p.n < 2:
            continue
        st, res, mask = served[t]
        assert matches_oracle(res, refs[t]), (t, p.n)
        assert np.array_equal(mask, refs[t]["mask"]), t


def test_request_larger_than_budget_rejected(aor):
    srv = aor.Server(hbm_budget_bytes=1 << 20, max_slots=4)
    p = synth.make_instance(50000, 1)
    with pytest.raises(aor.AorespError) as e:
        srv.submit(p.P, p.Q, aor.SolveParams(grid=256))
    assert e.value.status == aor.ENOMEM
    q = synth.make_instance(500, 2)
    rid = srv.submit(q.P, q.Q, aor.SolveParams(grid=64))
    st, res, mask = srv.poll(rid, timeout_us=-1)
    assert st in (aor.OK, aor.ENODATA)
    srv.close()


def test_poll_nonblocking_and_unknown_id(aor):
    srv = aor.Server()
    p = synth.make_instance(200000, 4)
    rid = srv.submit(p.P, p.Q, aor.SolveParams(grid=1024, angle_bins=3600))
    st, _, _ = srv.poll(rid, timeout_us=0)
    assert st in (aor.EBUSY, aor.OK)
    if st == aor.EBUSY:
        st, res, _ = srv.poll(rid, timeout_us=-1)
        assert st == aor.OK
    st, _, _ = srv.poll(123456789, timeout_us=0)
    assert st == aor.EINVAL
    srv.close()


def test_destroy_drains_queue(aor):
    srv = aor.Server(max_slots=2)
    ps = [synth.make_instance(5000, 70 + t) for t in range(6)]
    ids = [srv.submit(p.P, p.Q, aor.SolveParams(grid=128)) for p in ps]
    st, _, _ = srv.poll(ids[0], timeout_us=-1)
    assert st == aor.OK
    srv.close()   # the rest are drained before the loop exits


def test_served_options_equal_solo(aor):
    """Requests that mix the sampling rule, the angle gate and fine angle
    bins share batches; each served result equals its solo solve."""
    rng = np.random.default_rng(11)
    sizes = [int(x) for x in np.exp(rng.uniform(np.log(500), np.log(20000), 12))]
    probs = [synth.make_instance(n, 9500 + t, outlier_rate=0.85) for t, n in enumerate(sizes)]
    opts = [dict(vote_rule=t % 2, circle_samples=(0, 700, 2048)[t % 3], angle_gate=(t // 2) % 2,
                 angle_refine=(0, 8, 1)[t % 3]) for t in range(len(probs))]
    prms = [aor.SolveParams(angle_bins=360, **o) for o in opts]
    srv = aor.Server(hbm_budget_bytes=256 << 20, max_slots=6)
    ids = [srv.submit(p.P, p.Q, prm) for p, prm in zip(probs, prms)]
    served = [srv.poll(rid, timeout_us=-1) for rid in ids]
    srv.close()
    for t, (st, res, mask) in enumerate(served):
        r1, m1, st1 = aor.est_rotation(probs[t].P, probs[t].Q, prms[t])
        assert st == st1
        assert same(res, r1), (t, opts[t])
        assert res["angle_fine_bin"] == r1["angle_fine_bin"] and res["angle_fine_votes"] == r1["angle_fine_votes"]
        assert np.array_equal(mask, m1)
