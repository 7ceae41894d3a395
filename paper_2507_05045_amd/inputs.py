"""Seeded synthetic market-split instances.

This module is shared by the GPU path's tests and benchmark and by the
oracle's tests.  It only draws random numbers; it holds none of the solver's
arithmetic.

Instance family (Section 1, the hard family after Cornuejols and Dawande):
``n = 10 (m - 1)``, every ``a_ij`` uniform in ``[0, 99]`` and
``d_i = floor(sum_j a_ij / 2)``.  The paper's benchmark set (Section 4) is
drawn from the same family with ``a_ij`` in ``[0, K)``; the instances built
here stand in for it.

Generator (frozen; never change it silently, stored expected values depend
on it):

* ``A = default_rng(seed).integers(0, K, size=(m, n))`` as int32,
  ``d = A.sum(axis=1) // 2``;
* planted twin: ``x* = default_rng(seed + 10_000).integers(0, 2, size=n)``
  and ``d = A @ x*`` (so ``x*`` is a solution);
* stream of 512 instances: ``m = 5 + default_rng(0).integers(0, 4, 512)``,
  instance ``k`` uses seed ``1000 + k`` and is planted iff ``k`` is odd;
  arrival gaps are exponential draws from ``default_rng(7)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

PLANT_OFFSET = 10_000


@dataclass
class Instance:
    A: np.ndarray            # (m, n) int32, row-major
    d: np.ndarray            # (m,) int32
    name: str
    seed: int
    planted: Optional[np.ndarray] = None   # x* (uint8) when planted
    key_rows: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.A.shape[0])

    @property
    def n(self) -> int:
        return int(self.A.shape[1])


def make_matrix(m: int, n: int, seed: int, K: int = 100) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.integers(0, K, size=(m, n)).astype(np.int32))


def make_instance(m: int, n: int, seed: int, planted: bool = False, K: int = 100,
                  key_rows: int = 1,
                  accept: Optional[Callable[[np.ndarray], bool]] = None,
                  max_tries: int = 100_000) -> Instance:
    """Build one instance of the hard family.

    ``accept`` (planted only) lets a caller resample ``x*`` until a predicate
    holds, e.g. that ``x*`` lies in a residue slice; draws continue on the
    same generator so the result stays a function of ``seed``.
    """
    A = make_matrix(m, n, seed, K)
    kk = "" if K == 100 else f"_K{K}"
    if not planted:
        d = (A.astype(np.int64).sum(axis=1) // 2).astype(np.int32)
        return Instance(A, d, f"msp_{m}_{n}{kk}_s{seed}", seed, None, key_rows)
    rng = np.random.default_rng(seed + PLANT_OFFSET)
    for _ in range(max_tries):
        x = rng.integers(0, 2, size=n).astype(np.uint8)
        if accept is None or accept(x):
            break
    else:
        raise RuntimeError("no planted vector satisfied the predicate")
    d = (A.astype(np.int64) @ x.astype(np.int64)).astype(np.int32)
    return Instance(A, d, f"msp_{m}_{n}{kk}_s{seed}_planted", seed, x, key_rows)


def stream_instances(count: int = 512, base_seed: int = 1000) -> List[Instance]:
    """The uneven batched/served stream: m in {5,6,7,8}, n = 10(m-1),
    key rows r = m - 4, odd instances planted."""
    ms = 5 + np.random.default_rng(0).integers(0, 4, size=count)
    out = []
    for k in range(count):
        m = int(ms[k])
        inst = make_instance(m, 10 * (m - 1), base_seed + k, planted=bool(k & 1),
                             key_rows=m - 4)
        inst.meta["stream_index"] = k
        out.append(inst)
    return out


def poisson_arrivals(count: int, rate: float, seed: int = 7) -> np.ndarray:
    """Arrival times (seconds from 0) with exponential gaps at ``rate``/s."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=count)
    return np.cumsum(gaps) - gaps[0]


# Named workloads.  ``key_rows`` is the number of leading rows folded into the
# 1-D key (the surrogate constraint of Section 1).
CONFIGS = {
    "4_30": dict(m=4, n=30, key_rows=1, seeds=[0]),
    "6_50": dict(m=6, n=50, key_rows=1, seeds=[0]),
    "8_70": dict(m=8, n=70, key_rows=4, seeds=[0, 1, 2, 3, 4]),
    "9_80": dict(m=9, n=80, key_rows=4, seeds=[0]),
    "10_90": dict(m=10, n=90, key_rows=4, seeds=[0]),
}


def config_instances(name: str, planted_twin: bool = True) -> List[Instance]:
    c = CONFIGS[name]
    out = []
    for s in c["seeds"]:
        out.append(make_instance(c["m"], c["n"], s, False, key_rows=c["key_rows"]))
        if planted_twin:
            out.append(make_instance(c["m"], c["n"], s, True, key_rows=c["key_rows"]))
    return out


def random_small(m: int, n: int, seed: int, K: int = 100, zero_cols: int = 0,
                 planted: bool = True) -> Instance:
    """Small random instance for brute-force parity, optionally with forced
    all-zero columns (zero coefficients must still be enumerated, Section 3)."""
    inst = make_instance(m, n, seed, planted=planted, K=K)
    if zero_cols:
        rng = np.random.default_rng(seed + 77)
        cols = rng.choice(n, size=min(zero_cols, n), replace=False)
        A = inst.A.copy()
        A[:, cols] = 0
        x = inst.planted if inst.planted is not None else None
        if x is not None:
            d = (A.astype(np.int64) @ x.astype(np.int64)).astype(np.int32)
        else:
            d = (A.astype(np.int64).sum(axis=1) // 2).astype(np.int32)
        inst = Instance(np.ascontiguousarray(A), d, inst.name + f"_z{zero_cols}", seed, x)
    return inst
