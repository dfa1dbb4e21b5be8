"""Seeded synthetic inputs shaped like the paper's workloads.

The paper's experiments use points "randomly generated within a square" with
n = m (Section 5.1) and never state z.  This module draws such inputs and
nothing else: it contains none of the method's arithmetic, so both the HIP
path and the CPU oracle can be fed from it.

Recipe (fixed draw order per dataset: data x, y -> z noise -> queries):
  * coordinates are quantised to the 2^-20 lattice, x = floor(u * 2^20) / 2^20
    in [0, 1 - 2^-20], so they are exact in float32 and squared distances are
    exact in float64;
  * z = sin(6x) cos(6y) + 0.01 * N(0, 1), evaluated in float64 and rounded
    to float32 (that rounded value is the canonical input for both sides);
  * clustered data: 90 % from an isotropic Gaussian mixture (centres uniform
    in [0,1)^2, sigma = 0.02, equal weights; draws outside [0,1)^2 are
    redrawn) plus 10 % uniform background, then shuffled;
  * queries are uniform.

Named workloads (n data points, m queries, k neighbours):
  uniform_4k     n = m = 4096, uniform, k = 10, seed 1
  uniform_1m     n = m = 2^20, uniform, k = 10, seed 2
  clustered_256k n = m = 2^18, 16-component mixture, k = 15, seed 3
  batch_256      256 jobs, n log-uniform in [1024, 65536], m = n, k from {8, 10, 15},
                 jobs 0-127 uniform, 128-255 8-component mixture, seed 4000 + job
  learned_1m     n = m = 2^20, 16-component mixture, k = 15, seed 5 (training sets: seeds 100-103)
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

LATTICE = float(1 << 20)
LEVELS = (1.0, 2.0, 3.0, 4.0, 5.0)
R_MIN, R_MAX = 0.0, 2.0
OCCUPANCY = 2.0


def quantise(u: np.ndarray) -> np.ndarray:
    return (np.floor(u * LATTICE) / LATTICE).astype(np.float32)


def _uniform_xy(rng, n):
    x = quantise(rng.random(n))
    y = quantise(rng.random(n))
    return x, y


def _mixture_xy(rng, n, ncomp, sigma=0.02, background=0.10):
    ncl = n - int(round(background * n))
    centres = rng.random((ncomp, 2))
    px = np.empty(ncl)
    py = np.empty(ncl)
    filled = 0
    while filled < ncl:
        need = ncl - filled
        comp = rng.integers(0, ncomp, size=need)
        cx = centres[comp, 0] + sigma * rng.standard_normal(need)
        cy = centres[comp, 1] + sigma * rng.standard_normal(need)
        ok = (cx >= 0) & (cx < 1) & (cy >= 0) & (cy < 1)
        cnt = int(ok.sum())
        px[filled:filled + cnt] = cx[ok]
        py[filled:filled + cnt] = cy[ok]
        filled += cnt
    bx = rng.random(n - ncl)
    by = rng.random(n - ncl)
    ax = np.concatenate([px, bx])
    ay = np.concatenate([py, by])
    perm = rng.permutation(n)
    return quantise(ax[perm]), quantise(ay[perm])


def _field(rng, x, y):
    z = np.sin(6.0 * x.astype(np.float64)) * np.cos(6.0 * y.astype(np.float64))
    z = z + 0.01 * rng.standard_normal(x.size)
    return z.astype(np.float32)


@dataclass
class Dataset:
    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    qx: np.ndarray
    qy: np.ndarray
    k: int
    seed: int
    levels: tuple = LEVELS
    r_min: float = R_MIN
    r_max: float = R_MAX
    occupancy: float = OCCUPANCY
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.x.size)

    @property
    def m(self):
        return int(self.qx.size)


def make(n, m, k, seed, kind="uniform", ncomp=16, name=None):
    """One dataset: data (uniform or mixture), z field, uniform queries."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        x, y = _uniform_xy(rng, n)
    elif kind == "mixture":
        x, y = _mixture_xy(rng, n, ncomp)
    else:
        raise ValueError(kind)
    z = _field(rng, x, y)
    qx, qy = _uniform_xy(rng, m)
    return Dataset(name or "%s_%d_%d" % (kind, n, m), x, y, z, qx, qy, k, seed, meta=dict(kind=kind, ncomp=ncomp))


def sample_queries(m, count, seed):
    """Sorted sample of query indices (its own generator, seeded seed + 1000)."""
    rng = np.random.default_rng(seed + 1000)
    count = min(count, m)
    return np.sort(rng.choice(m, size=count, replace=False)).astype(np.int64)


def uniform_4k():
    return make(4096, 4096, 10, 1, "uniform", name="uniform_4k")


def uniform_1m():
    return make(1 << 20, 1 << 20, 10, 2, "uniform", name="uniform_1m")


def clustered_256k():
    return make(1 << 18, 1 << 18, 15, 3, "mixture", 16, name="clustered_256k")


def learned_1m():
    return make(1 << 20, 1 << 20, 15, 5, "mixture", 16, name="learned_1m")


def learned_training_sets(n=1 << 20, queries_per_set=50_000, seeds=(100, 101, 102, 103)):
    """Held-out datasets for training the learned-R network (mixture recipe, uniform queries)."""
    return [make(n, queries_per_set, 15, s, "mixture", 16, name="train_%d" % s) for s in seeds]


def batch_jobs(count=256, base_seed=4000, n_lo=1024, n_hi=65536):
    """Independent jobs of uneven size: n log-uniform in [n_lo, n_hi], m = n, k from {8, 10, 15}."""
    jobs = []
    for j in range(count):
        rng = np.random.default_rng(base_seed + j)
        n = int(np.floor(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi + 1)))))
        n = max(n_lo, min(n_hi, n))
        k = int(rng.choice([8, 10, 15]))
        kind = "uniform" if j < count // 2 else "mixture"
        jobs.append(make(n, n, k, base_seed + j + 100000, kind, 8, name="job%03d" % j))
    return jobs


WORKLOADS = {
    "uniform_4k": uniform_4k,
    "uniform_1m": uniform_1m,
    "clustered_256k": clustered_256k,
    "learned_1m": learned_1m,
}
