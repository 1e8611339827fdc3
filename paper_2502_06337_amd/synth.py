"""Seeded synthetic correspondence generator (inputs only).

This module draws the point sets of the problem statement (Sec. I, Eq. (1)):
inliers satisfy q_i = R p_i + eps_i, outliers are unrelated points.  It is the
only code shared by the oracle side and the HIP side of the tests and of the
benchmark, and it holds none of the estimation method's arithmetic: no
projection, no voting, no histogram, no Rodrigues step.

Workload shape follows the synthetic experiments (Sec. V-A): noise sigma =
0.01, a fraction rho of outliers drawn as random points.  The point cloud is
uniform in [-1, 1)^3 (the paper normalises x to unit length; that variant is
``unit_p=True``).

Random numbers come from SplitMix64 (Steele, Lea, Flood 2014), used as a
counter-based generator: draw k of stream s is mix(key(seed, s) + (k+1)*gamma).
  * float32 uniform in [0, 1): (x >> 40) * 2**-24   (exact)
  * float64 uniform in [0, 1): (x >> 11) * 2**-53
  * standard normal: Box-Muller in float64
  * rotation: Shoemake's uniform unit quaternion
  * inlier positions: a uniform permutation (sort of random 64-bit keys)
Outputs are SoA float32 arrays of shape (3, n): row 0 = x, row 1 = y, row 2 = z.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream ids
_S_P, _S_Q, _S_NOISE, _S_ROT, _S_PERM, _S_META = 1, 2, 3, 4, 5, 6


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        base = np.array([(int(seed) * 0x100 + stream) & 0xFFFFFFFFFFFFFFFF],
                        dtype=np.uint64)
        return _mix(base + _GAMMA)[0]


def raw64(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """`count` SplitMix64 outputs of (seed, stream), starting at draw `offset`."""
    k = _key(seed, stream)
    idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(k + idx * _GAMMA)


def uniform_f32(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    x = raw64(seed, stream, count, offset)
    return (x >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)


def uniform_f64(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    x = raw64(seed, stream, count, offset)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal_f64(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    u = uniform_f64(seed, stream, 2 * count, 2 * offset)
    u1 = 1.0 - u[0::2]  # (0, 1]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def random_rotation(seed: int, which: int = 0) -> np.ndarray:
    """Uniform rotation on SO(3) from Shoemake's quaternion, float64 3x3."""
    u1, u2, u3 = uniform_f64(seed, _S_ROT, 3, 3 * which)
    s1, s2 = math.sqrt(1.0 - u1), math.sqrt(u1)
    x = s1 * math.sin(2 * math.pi * u2)
    y = s1 * math.cos(2 * math.pi * u2)
    z = s2 * math.sin(2 * math.pi * u3)
    w = s2 * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ], dtype=np.float64)


@dataclass
class Instance:
    P: np.ndarray                # (3, n) float32
    Q: np.ndarray                # (3, n) float32
    R_gt: list                   # list of (3, 3) float64 ground-truth rotations
    labels: np.ndarray           # (n,) int8: 0 = outlier, t+1 = inlier of rotation t
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.P.shape[1])


def make_instance(n: int, seed: int, outlier_rate: float = 0.9, sigma: float = 0.01,
                  n_rot: int = 1, inlier_frac_each: float | None = None,
                  unit_p: bool = False) -> Instance:
    """One synthetic problem.

    n_rot == 1: round(n * (1 - outlier_rate)) inliers of one rotation.
    n_rot > 1 : each rotation owns round(n * inlier_frac_each) inliers; the rest
                are outliers (e.g. 3 x 10% + 70% outliers).
    """
    n = int(n)
    if n_rot == 1:
        counts = [int(round(n * (1.0 - outlier_rate)))]
    else:
        f = inlier_frac_each if inlier_frac_each is not None else (1.0 - outlier_rate) / n_rot
        counts = [int(round(n * f))] * n_rot
    if sum(counts) > n:
        raise ValueError("inlier counts exceed n")

    P = (2.0 * uniform_f32(seed, _S_P, 3 * n) - 1.0).astype(np.float32).reshape(3, n)
    if unit_p:
        nrm = np.sqrt((P.astype(np.float64) ** 2).sum(axis=0))
        nrm[nrm == 0] = 1.0
        P = (P / nrm).astype(np.float32)
    Q = (2.0 * uniform_f32(seed, _S_Q, 3 * n) - 1.0).astype(np.float32).reshape(3, n)

    keys = raw64(seed, _S_PERM, n)
    perm = np.argsort(keys, kind="stable")
    labels = np.zeros(n, dtype=np.int8)
    Rs = []
    start = 0
    noise = normal_f64(seed, _S_NOISE, 3 * n).reshape(3, n)
    for t, cnt in enumerate(counts):
        R = random_rotation(seed, t)
        Rs.append(R)
        idx = perm[start:start + cnt]
        start += cnt
        labels[idx] = t + 1
        qi = R @ P[:, idx].astype(np.float64) + sigma * noise[:, idx]
        Q[:, idx] = qi.astype(np.float32)
    return Instance(P=np.ascontiguousarray(P), Q=np.ascontiguousarray(Q), R_gt=Rs,
                    labels=labels, seed=seed,
                    meta={"n": n, "outlier_rate": outlier_rate, "sigma": sigma,
                          "n_rot": n_rot, "inlier_counts": counts})


def config_seed(config: int, t: int) -> int:
    """Instance t of workload configuration c uses seed 1000*c + t."""
    return 1000 * config + t


def batch_instances(count: int, seed: int, n_lo: float = 1e3, n_hi: float = 1e5,
                    rho_lo: float = 0.5, rho_hi: float = 0.95,
                    sig_lo: float = 0.001, sig_hi: float = 0.02) -> list[Instance]:
    """Many independent problems: n log-uniform, outlier rate and sigma uniform."""
    u = uniform_f64(seed, _S_META, 3 * count).reshape(count, 3)
    out = []
    for t in range(count):
        n = int(round(math.exp(math.log(n_lo) + u[t, 0] * (math.log(n_hi) - math.log(n_lo)))))
        rho = rho_lo + u[t, 1] * (rho_hi - rho_lo)
        sig = sig_lo + u[t, 2] * (sig_hi - sig_lo)
        out.append(make_instance(n, seed * 100003 + t, outlier_rate=rho, sigma=sig))
    return out


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process: exponential inter-arrival gaps."""
    expect = int(rate * duration * 1.5) + 64
    u = uniform_f64(seed, _S_META, expect)
    gaps = -np.log(1.0 - u) / rate
    t = np.cumsum(gaps)
    return t[t < duration]


def log_uniform_sizes(count: int, seed: int, lo: float, hi: float) -> np.ndarray:
    u = uniform_f64(seed, _S_META, count, offset=1 << 20)
    return np.rint(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)
