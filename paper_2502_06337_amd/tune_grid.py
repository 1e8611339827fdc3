#!/usr/bin/env python3
"""Offline autotuner of the coarse grid resolution G per problem size.

For every size bucket b (n in [2^b, 2^(b+1))) it solves a set of seeded
synthetic problems shaped like the batched workload (outlier rate uniform in
[0.5, 0.95], noise sigma uniform in [0.001, 0.02], 360 angle bins, no
refinement) at each candidate G in {128, 256, 512, 1024} on the GPU, and
records for each G the rotation error against the generating rotation and the
batch's solve time.  A candidate's loss is the mean error with every error
capped at 5 degrees (a failed detection costs 5 degrees, however wrong).  The
chosen G of a bucket is the smallest one whose loss is within 25% of the best
candidate's (a finer grid costs about twice the time per step of G for a
loss that differs by 10-20% between neighbouring candidates), and the table is
made non-decreasing in n (a larger problem never gets a coarser grid).

Writes the sweep (every score) as JSON and the table the library compiles in
(csrc/grid_table.inc): aoresp_grid_for_n(n) looks n's bucket up there, so G
stays a pure function of n and every solve records it in result.grid.

Usage (on a GPU): python -m paper_2502_06337_amd.tune_grid --out DIR [--count K]
         python -m paper_2502_06337_amd.tune_grid --out DIR --rescore DIR/grid_table.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

CANDIDATES = (128, 256, 512, 1024)
BUCKETS = range(9, 21)          # n from 512 to 2^21 - 1; outside, the nearest bucket
FAIL_DEG = 5.0
LOSS_TOL = 1.25
TABLE_VERSION = 1


def rotation_error_deg(R_true, R_est) -> float:
    c = (np.trace(np.asarray(R_true, np.float64).T @ np.asarray(R_est, np.float64)) - 1.0) / 2.0
    return float(np.degrees(np.arccos(np.clip(c, -1.0, 1.0))))


def sweep_bucket(aor, synth, torch, b: int, count: int) -> dict:
    u = synth.uniform_f64(40000 + b, 0, 3 * count).reshape(count, 3)
    insts = []
    for t in range(count):
        n = int(round(2.0 ** (b + u[t, 0])))            # log-uniform inside the bucket
        rho = 0.5 + 0.45 * u[t, 1]
        sig = 0.001 + 0.019 * u[t, 2]
        insts.append(synth.make_instance(n, 41000 + 1000 * b + t, outlier_rate=rho, sigma=sig))
    sizes = [i.n for i in insts]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    dev = torch.device("cuda:0")
    P = torch.from_numpy(np.concatenate([i.P for i in insts], axis=1)).to(dev)
    Q = torch.from_numpy(np.concatenate([i.Q for i in insts], axis=1)).to(dev)
    scores = {}
    for G in CANDIDATES:
        prm = aor.SolveParams(grid=G, angle_bins=360)
        outs, _, _ = aor.est_rotation_batch(P, Q, off, prm, want_mask=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            aor.est_rotation_batch(P, Q, off, prm, want_mask=False)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 3
        errs = np.array([rotation_error_deg(i.R_gt[0], o["R"]) for i, o in zip(insts, outs)])
        scores[G] = {"loss_deg": float(np.minimum(errs, FAIL_DEG).mean()), "median_deg": float(np.median(errs)),
                     "failures": int((errs > FAIL_DEG).sum()), "p90_deg": float(np.percentile(errs, 90)),
                     "batch_ms": dt * 1e3}
    return {"bucket": b, "n_range": [2 ** b, 2 ** (b + 1) - 1], "count": count, "total_n": int(off[-1]),
            "scores": {str(G): s for G, s in scores.items()}, "grid": choose(scores)}


def choose(scores: dict) -> int:
    """Smallest G whose capped mean error is within 25% of the best one's."""
    best = min(s["loss_deg"] for s in scores.values())
    return min(int(G) for G, s in scores.items() if s["loss_deg"] <= LOSS_TOL * best)


def write_table(rows: list, out_dir: str) -> None:
    rows = sorted(rows, key=lambda r: r["bucket"])
    first = rows[0]["bucket"]
    grids = list(np.maximum.accumulate([r["grid"] for r in rows]))
    for r, g in zip(rows, grids):
        r["table_grid"] = int(g)
    lines = [
        "// Coarse grid resolution per size bucket b = floor(log2 n), written by",
        "// paper_2502_06337_amd/tune_grid.py from its sweep of rotation error and",
        "// solve time on seeded batched-workload problems (grid_table.json holds",
        "// every score).  Buckets below the first or above the last use the",
        "// nearest entry.",
        f"constexpr int kGridTableVersion = {TABLE_VERSION};",
        f"constexpr int kGridTableFirst = {first};",
        f"constexpr int kGridTable[{len(grids)}] = {{{', '.join(str(g) for g in grids)}}};",
        "",
    ]
    with open(os.path.join(out_dir, "grid_table.inc"), "w") as f:
        f.write("\n".join(lines))
    with open(os.path.join(out_dir, "grid_table.json"), "w") as f:
        json.dump({"version": TABLE_VERSION, "candidates": list(CANDIDATES), "fail_deg": FAIL_DEG,
                   "rule": f"smallest G whose mean error (capped at fail_deg) is within a factor {LOSS_TOL} "
                           "of the best; then non-decreasing in n",
                   "buckets": rows}, f, indent=1)
        f.write("\n")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True, help="directory for grid_table.json and grid_table.inc")
    ap.add_argument("--count", type=int, default=128, help="problems per bucket (48 at most above n = 2^17)")
    ap.add_argument("--rescore", metavar="JSON", help="choose again from a stored sweep (no GPU needed)")
    args = ap.parse_args()
    if args.rescore:
        with open(args.rescore) as f:
            rows = json.load(f)["buckets"]
        for r in rows:
            r["grid"] = choose(r["scores"])
        os.makedirs(args.out, exist_ok=True)
        write_table(rows, args.out)
        return 0
    import torch
    import paper_2502_06337_amd as aor
    from paper_2502_06337_amd import synth
    if not torch.cuda.is_available():
        print("tune_grid: no GPU visible", file=sys.stderr)
        return 1
    aor.load_library()
    os.makedirs(args.out, exist_ok=True)
    rows = []
    for b in BUCKETS:
        count = args.count if b < 17 else min(args.count, 48)
        r = sweep_bucket(aor, synth, torch, b, count)
        rows.append(r)
        print(f"bucket {b}: G = {r['grid']} "
              + " ".join(f"{G}:{s['failures']}/{s['loss_deg']:.3f}/{s['median_deg']:.3f}/{s['batch_ms']:.2f}ms"
                         for G, s in r["scores"].items()), flush=True)
    write_table(rows, args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
