"""The request loop's scheduler on the CPU, with a fake executor and a fake
clock (tests/fake_sched.cpp): admission under the device-memory budget
counting the pipelines' cached buffers, arrival order, slot limits,
deadlines while queued and in a batch, device errors and allocation
failures (retried at the exact size, else reported as ENOMEM)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
OK, ENOMEM, EDEVICE, ENODATA, EBUSY, ETIMEDOUT = 0, -2, -3, -4, -5, -6


@pytest.fixture(scope="module")
def fs(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("fakesched") / "libfakesched.so")
    r = subprocess.run([gxx, "-O1", "-std=c++17", "-shared", "-fPIC", os.path.join(HERE, "fake_sched.cpp"),
                        "-o", out, "-lpthread"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    L = C.CDLL(out)
    L.fs_create.restype = C.c_void_p
    L.fs_create.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32]
    L.fs_destroy.argtypes = [C.c_void_p]
    L.fs_submit.restype = C.c_uint64
    L.fs_submit.argtypes = [C.c_void_p, C.c_uint64]
    L.fs_step.argtypes = [C.c_void_p]
    L.fs_advance.argtypes = [C.c_void_p, C.c_int64]
    L.fs_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_uint32)]
    for f in ("fs_max_total", "fs_peak_held"):
        getattr(L, f).restype = C.c_uint64
        getattr(L, f).argtypes = [C.c_void_p]
    L.fs_held.restype = C.c_uint64
    L.fs_held.argtypes = [C.c_void_p, C.c_int]
    L.fs_launches.argtypes = [C.c_void_p]
    L.fs_releases.argtypes = [C.c_void_p]
    L.fs_order.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.c_int]
    L.fs_set.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int64]
    L.fs_stats.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
    return L


class H:
    """One scheduler with a fake executor (100 device bytes per correspondence
    + 64 per request; batches take step_us of fake time)."""

    def __init__(self, L, budget, slots=256, timeout=0, step_us=1000):
        self.L, self.h = L, L.fs_create(budget, slots, timeout)
        L.fs_set(self.h, 0, 0, 0, step_us)
        self.budget = budget

    def submit(self, n):
        return self.L.fs_submit(self.h, n)

    def poll(self, rid):
        v = C.c_uint32(0)
        st = self.L.fs_poll(self.h, rid, C.byref(v))
        return st, v.value

    def run(self, ids, max_iter=10000):
        """Step and advance the clock until every id has finished."""
        res = {}
        for _ in range(max_iter):
            self.L.fs_step(self.h)
            assert self.L.fs_max_total(self.h) <= self.budget
            for rid in ids:
                if rid not in res:
                    st, v = self.poll(rid)
                    if st != EBUSY:
                        res[rid] = (st, v)
            if len(res) == len(ids):
                return res
            self.L.fs_advance(self.h, 100)
        raise AssertionError("requests did not finish")

    def order(self):
        buf = (C.c_uint64 * 4096)()
        k = self.L.fs_order(self.h, buf, 4096)
        return list(buf[:k])

    def close(self):
        self.L.fs_destroy(self.h)


def grown(need):
    return need + need // 4 + 256


def test_admission_stays_within_budget(fs):
    # two requests of 1000 correspondences do not fit one grown pipeline
    budget = 250_000
    h = H(fs, budget)
    ids = [h.submit(1000) for _ in range(6)]
    res = h.run(ids)
    assert all(st == OK and v == 1000 for st, v in res.values())
    assert fs.fs_max_total(h.h) <= budget
    assert fs.fs_peak_held(h.h) <= budget
    assert h.order() == ids                      # arrival order
    h.close()


def test_slots_and_order(fs):
    h = H(fs, 1 << 40, slots=3)
    ids = [h.submit(10 + t) for t in range(10)]
    res = h.run(ids)
    assert h.order() == ids
    assert fs.fs_launches(h.h) == 4              # batches of 3, 3, 3, 1
    assert all(st == OK for st, _ in res.values())
    h.close()


def test_small_requests_are_enodata(fs):
    h = H(fs, 1 << 30)
    ids = [h.submit(0), h.submit(1), h.submit(2)]
    res = h.run(ids)
    assert [res[i][0] for i in ids] == [ENODATA, ENODATA, OK]
    h.close()


def test_request_alone_over_budget_is_refused(fs):
    h = H(fs, 100_000)
    assert h.submit(2000) == 0                   # 200 kB alone
    assert h.submit(500) != 0
    h.close()


def test_deadline_while_queued_and_in_batch(fs):
    # one slot, batches of 8 ms, deadlines 5 ms after submit
    h = H(fs, 1 << 30, slots=1, timeout=5000, step_us=8000)
    ids = [h.submit(100) for _ in range(3)]
    res = h.run(ids)
    # two ran (one per pipeline) but finished after their deadlines; the third expired queued
    assert [res[i][0] for i in ids] == [ETIMEDOUT] * 3
    assert fs.fs_launches(h.h) == 2
    h.close()
    # batches of 2 ms meet the deadline
    h = H(fs, 1 << 30, slots=4, timeout=5000, step_us=2000)
    ids = [h.submit(100) for _ in range(4)]
    res = h.run(ids)
    assert all(res[i][0] == OK for i in ids)
    h.close()


def test_device_error_fails_only_its_batch(fs):
    h = H(fs, 1 << 30, slots=2)
    fs.fs_set(h.h, 0, 0, 1, 1000)
    ids = [h.submit(100) for _ in range(6)]
    res = h.run(ids)
    sts = [res[i][0] for i in ids]
    assert sts[:2] == [EDEVICE, EDEVICE]
    assert sts[2:] == [OK] * 4
    h.close()


def test_allocation_failure_is_retried_exactly(fs):
    h = H(fs, 1 << 30)
    fs.fs_set(h.h, 1, 0, 0, 1000)                # the first growth fails once
    ids = [h.submit(1000) for _ in range(3)]
    res = h.run(ids)
    assert all(st == OK for st, _ in res.values())
    h.close()
    h = H(fs, 1 << 30)
    fs.fs_set(h.h, 0, 1, 0, 1000)                # every allocation fails
    ids = [h.submit(1000) for _ in range(3)]
    res = h.run(ids)
    assert all(st == ENOMEM for st, _ in res.values())
    h.close()


def test_cached_buffers_count_against_budget(fs):
    """A large request leaves its pipeline's buffers large; a later small one
    on the other pipeline fits only once that idle cache is released."""
    need_big = 2000 * 100 + 64
    budget = grown(need_big) + 50_000
    h = H(fs, budget)
    big = h.submit(2000)
    h.run([big])
    assert fs.fs_held(h.h, 0) + fs.fs_held(h.h, 1) == grown(need_big)
    small = h.submit(500)
    res = h.run([small])
    assert res[small][0] == OK
    assert fs.fs_releases(h.h) >= 1
    assert fs.fs_max_total(h.h) <= budget
    h.close()


def test_latency_stats(fs):
    h = H(fs, 1 << 30, slots=1, step_us=1000)
    ids = [h.submit(100) for _ in range(4)]
    h.run(ids)
    p50, p99, done = C.c_double(), C.c_double(), C.c_uint64()
    fs.fs_stats(h.h, C.byref(p50), C.byref(p99), C.byref(done))
    assert done.value == 4
    # one request per batch, two pipelines, 1 ms per batch: latencies 1, 1, 2, 2 ms
    assert 900 <= p50.value <= 2100 and 1900 <= p99.value <= 2200
    h.close()
