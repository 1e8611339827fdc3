#!/usr/bin/env python3
"""Writes the stored expected values of the paper-scale parity tests.

Calls only the CPU oracle (and the seeded input generator).  The coarse
accumulator at n = 10^6, G = 1024 costs about 5000 core-seconds by the
oracle's brute force, so it is computed over column chunks of (P, Q) in
threads (the oracle releases the interpreter lock while it runs) and the chunk
grids are summed: the accumulator is additive over correspondences (pinned in
the oracle's tests).  Everything after the coarse grid is the oracle's own
single-threaded code.

Stored per workload (JSON, one file each):
  - the coarse grid as a sha256 digest of each row (little-endian uint32) and
    the total of all votes;
  - the peak(s) (Sec. IV-A; Sec. IV-D for several rotations), and per peak
    the refinement grid's row digests, the angle histogram's digest and the
    whole result (cells, votes, the bit patterns of the axis (Eq. (8)), the
    angle and R (Eq. (2)), the inlier count and a digest of the mask).

Usage: python tests/golden/make_goldens.py c2|c3 [--threads T]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2502_06337_amd import synth  # noqa: E402

WORKLOADS = {
    # plain single solve at paper scale (Sec. V-A synthetic setup: 10^6 points, 90% outliers)
    "c2": dict(n=1_000_000, seed=2000, n_rot=1, outlier_rate=0.9, G=1024, M=64, w=1, B=3600, tau=0.05, k=1, rad=5),
    # three rotations, 10% inliers each, 70% outliers (Sec. V-B multi-rotation setup)
    "c3": dict(n=1_000_000, seed=3000, n_rot=3, outlier_rate=0.7, G=1024, M=64, w=1, B=3600, tau=0.05, k=3, rad=5),
}


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u4").tobytes()).hexdigest()[:16]


def row_digests(g) -> list:
    return [digest(row) for row in np.asarray(g)]


def make_input(wl: dict):
    if wl["n_rot"] == 1:
        return synth.make_instance(wl["n"], wl["seed"], outlier_rate=wl["outlier_rate"], sigma=0.01)
    return synth.make_instance(wl["n"], wl["seed"], n_rot=wl["n_rot"], inlier_frac_each=0.1, sigma=0.01)


def coarse_grid_chunked(P, Q, G: int, threads: int, chunks: int = 64):
    n = P.shape[1]
    bounds = np.linspace(0, n, chunks + 1).astype(np.int64)
    parts = [(int(bounds[i]), int(bounds[i + 1])) for i in range(chunks)]
    total = np.zeros((G, G), np.uint64)
    done = 0
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for g in ex.map(lambda ab: oracle.coarse_grid(P[:, ab[0]:ab[1]], Q[:, ab[0]:ab[1]], G), parts):
            total += g
            done += 1
            print(f"  coarse chunk {done}/{chunks} ({time.time() - t0:.0f} s)", flush=True)
    assert total.max() < 2 ** 32
    return total.astype(np.uint32)


def result_record(r: dict) -> dict:
    rec = {k: int(r[k]) for k in ("peak_cell", "axis_votes", "fine_cell", "fine_votes", "angle_bin",
                                  "angle_votes", "n_inliers", "grid")}
    rec["axis_bits"] = [int(x) for x in np.asarray(r["axis"], np.float32).view(np.uint32)]
    rec["angle_bits"] = int(np.float32(r["angle"]).view(np.uint32))
    rec["R_bits"] = [int(x) for x in np.asarray(r["R"], np.float32).ravel().view(np.uint32)]
    rec["mask_sha256"] = hashlib.sha256(np.ascontiguousarray(r["mask"], np.uint8).tobytes()).hexdigest()[:16]
    return rec


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(WORKLOADS))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    wl = WORKLOADS[args.workload]
    oracle.lib()
    inst = make_input(wl)
    P, Q = inst.P, inst.Q
    G, M, w, B, tau = wl["G"], wl["M"], wl["w"], wl["B"], wl["tau"]
    print(f"{args.workload}: coarse grid G={G} over n={P.shape[1]} with {args.threads} threads", flush=True)
    grid = coarse_grid_chunked(P, Q, G, args.threads)
    if wl["k"] == 1:
        peak, votes = oracle.argmax(grid)
        peaks = [(peak, votes)]
    else:
        peaks = oracle.topk_peaks(grid, wl["k"], wl["rad"])
    results = []
    for peak, votes in peaks:
        print(f"  finishing peak {peak} ({votes} votes)", flush=True)
        r = oracle.finish_peak(P, Q, G, M, w, B, tau, peak, votes, want_grids=True)
        rec = result_record(r)
        rec["fine_rows"] = row_digests(r["fine"])
        rec["hist_sha256"] = digest(r["hist"])
        results.append(rec)
    out = {
        "workload": args.workload,
        "what": "stored oracle outputs for the paper-scale parity tests; written by tests/golden/make_goldens.py "
                "from the CPU oracle only",
        "params": wl,
        "coarse_sum": int(grid.astype(np.uint64).sum()),
        "coarse_rows": row_digests(grid),
        "peaks": [[int(c), int(v)] for c, v in peaks],
        "results": results,
    }
    path = os.path.join(HERE, f"{args.workload}_seed{wl['seed']}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
