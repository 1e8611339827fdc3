"""The oracle's coarse accumulator over column chunks in threads (the oracle's
C code runs without the interpreter lock), summed: the accumulator is additive
over correspondences, which the oracle's pins check.  Test helper only."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def coarse_grid(orc, P, Q, G: int, threads: int = 0) -> np.ndarray:
    threads = threads or min(16, os.cpu_count() or 1)
    n = P.shape[1]
    chunks = max(1, min(4 * threads, n // 64))
    b = np.linspace(0, n, chunks + 1).astype(np.int64)
    parts = [(int(b[i]), int(b[i + 1])) for i in range(chunks) if b[i + 1] > b[i]]
    total = np.zeros((G, G), np.uint64)
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for g in ex.map(lambda ab: orc.coarse_grid(P[:, ab[0]:ab[1]], Q[:, ab[0]:ab[1]], G), parts):
            total += g
    return total.astype(np.uint32)
