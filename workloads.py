"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method (no random-number generator of the
method, no point map, no action, no sums): it only builds input descriptions --
lattice parameters, boxes, subvolume lists with heap ids, per-subvolume sample
counts and offsets, and request streams for the serving workload.  Both the HIP
path and the CPU oracle consume what it produces.

Workloads (sizes of the paper's own run, section 4: a 10x2 lattice; the other
shapes widen it):
  * ``burgers4x2``   4x2 lattice, nu=1, D=1, box [-4,4]^8, 2^20 points, 16 subvolumes
  * ``burgers10x2``  10x2 lattice, nu=1, D=1, box [-4,4]^20, 2^30 points, 1024 subvolumes
  * ``burgers16x4``  16x4 lattice, nu=0.5, D=1, box [-3,3]^64, 2^34 points, 4096 subvolumes
  * ``adaptive10x2`` 10x2 lattice, nu in {0.1, 0.5, 1}, start partition of 1024 at 2^12
  * serving: Poisson arrivals (200/s) with lattice, nu, budget drawn per request
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    nt: int
    nu: float
    D: float
    box: float          # box is [-box, box]^d
    split_log2: int     # 2^split_log2 equal subvolumes
    budget: int         # total number of samples
    seed: int = 1
    a: float = 1.0
    tau: float = 1.0

    @property
    def d(self) -> int:
        return self.nx * self.nt

    @property
    def n_sub(self) -> int:
        return 1 << self.split_log2


WORKLOADS = {
    "burgers4x2": Workload("burgers4x2", 4, 2, 1.0, 1.0, 4.0, 4, 1 << 20),
    "burgers10x2": Workload("burgers10x2", 10, 2, 1.0, 1.0, 4.0, 10, 1 << 30),
    "burgers16x4": Workload("burgers16x4", 16, 4, 0.5, 1.0, 3.0, 12, 1 << 34),
}


def scaled(w: Workload, budget: int, split_log2: int | None = None) -> Workload:
    """The same lattice and box with a different budget (and split)."""
    return dataclasses.replace(w, budget=int(budget),
                               split_log2=w.split_log2 if split_log2 is None else split_log2)


@dataclasses.dataclass
class SubvolumeList:
    """Subvolumes as the library and the oracle take them: heap ids, boxes
    (row-major n x d), sample counts and first sample index of each."""
    ids: np.ndarray      # uint64
    lo: np.ndarray       # float64 (n, d)
    hi: np.ndarray       # float64 (n, d)
    n: np.ndarray        # uint64
    offset: np.ndarray   # uint64

    def __len__(self) -> int:
        return int(self.ids.shape[0])

    def subset(self, idx) -> "SubvolumeList":
        idx = np.asarray(idx, dtype=np.int64)
        return SubvolumeList(self.ids[idx].copy(), self.lo[idx].copy(), self.hi[idx].copy(),
                             self.n[idx].copy(), self.offset[idx].copy())


def _bisect(lo, hi, dim):
    mid = 0.5 * (lo[dim] + hi[dim])
    lo_a, hi_a = lo.copy(), hi.copy()
    lo_b, hi_b = lo.copy(), hi.copy()
    hi_a[dim] = mid
    lo_b[dim] = mid
    return (lo_a, hi_a), (lo_b, hi_b)


def uniform_partition(d: int, box: float, split_log2: int, per_sub: int | np.ndarray,
                      offset: int = 0) -> SubvolumeList:
    """2^split_log2 subvolumes of [-box, box]^d, bisecting dims 0, 1, ... in turn
    (dim t mod d at level t); heap ids 2^k .. 2^(k+1)-1 in increasing order."""
    leaves = [(1, np.full(d, -float(box)), np.full(d, float(box)))]
    for t in range(split_log2):
        nxt = []
        for hid, lo, hi in leaves:
            (la, ha), (lb, hb) = _bisect(lo, hi, t % d)
            nxt += [(2 * hid, la, ha), (2 * hid + 1, lb, hb)]
        leaves = nxt
    return _as_list(leaves, per_sub, offset)


def random_partition(d: int, box: float, n_leaves: int, per_sub, seed: int,
                     offset=0) -> SubvolumeList:
    """An uneven bisection tree: repeatedly halve a random leaf along a random
    dimension (numpy PCG64(seed)).  Leaves are returned in increasing id order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    leaves = [(1, np.full(d, -float(box)), np.full(d, float(box)))]
    while len(leaves) < n_leaves:
        j = int(rng.integers(len(leaves)))
        hid, lo, hi = leaves.pop(j)
        (la, ha), (lb, hb) = _bisect(lo, hi, int(rng.integers(d)))
        leaves += [(2 * hid, la, ha), (2 * hid + 1, lb, hb)]
    leaves.sort(key=lambda t: t[0])
    return _as_list(leaves, per_sub, offset)


def _as_list(leaves, per_sub, offset) -> SubvolumeList:
    ns = len(leaves)
    ids = np.array([t[0] for t in leaves], dtype=np.uint64)
    lo = np.stack([t[1] for t in leaves]).astype(np.float64)
    hi = np.stack([t[2] for t in leaves]).astype(np.float64)
    n = np.ascontiguousarray(np.broadcast_to(np.asarray(per_sub, dtype=np.uint64), (ns,)))
    off = np.ascontiguousarray(np.broadcast_to(np.asarray(offset, dtype=np.uint64), (ns,)))
    return SubvolumeList(ids, lo, hi, n.copy(), off.copy())


def log_uniform_counts(ns: int, lo_log2: int, hi_log2: int, seed: int) -> np.ndarray:
    """Per-subvolume sample counts 2^U(lo, hi), rounded to integers (uneven work)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.uniform(lo_log2, hi_log2, size=ns)
    return np.maximum(2, np.round(2.0 ** e)).astype(np.uint64)


@dataclasses.dataclass(frozen=True)
class Request:
    index: int
    arrival_s: float
    nx: int
    nt: int
    nu: float
    D: float
    box: float
    budget: int
    seed: int
    split_log2: int = 4


SERVING_SHAPES = ((4, 2), (8, 2), (10, 2), (16, 4))


def serving_requests(rate_hz: float, duration_s: float, seed: int = 1,
                     budget_log2=(16, 26)) -> list[Request]:
    """Poisson arrivals; lattice uniform over 4x2, 8x2, 10x2, 16x4; nu log-uniform
    in [0.05, 2]; D = 1; budget 2^U(16, 26) rounded to a multiple of 16; box
    [-4, 4] for two time slices and [-3, 3] for 16x4; Philox seed = index + 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out, t, i = [], 0.0, 0
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        nx, nt = SERVING_SHAPES[int(rng.integers(len(SERVING_SHAPES)))]
        nu = float(math.exp(rng.uniform(math.log(0.05), math.log(2.0))))
        budget = int(round(2.0 ** rng.uniform(*budget_log2) / 16.0)) * 16
        box = 3.0 if (nx, nt) == (16, 4) else 4.0
        out.append(Request(i, t, nx, nt, nu, 1.0, box, max(budget, 64), i + 1))
        i += 1
    return out
