"""Seeded synthetic inputs for the FE-P3M hot path.

This module only draws positions and charges; it contains none of the
method's arithmetic, so both the oracle (tests) and the GPU path (bench,
smoke, tests) can use it without sharing any computation.

The workloads follow the paper's own test problems, which are random
charges in a triply periodic unit cube (Section 4), plus the sizes this
build measures: uniform random charges at three sizes, a clustered
distribution that skews element occupancy, a batch of independent
configurations of uneven size, and the paper's two biased sub-cubes.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    N: int
    n: int                 # elements per axis
    L: float = 1.0
    kind: str = "uniform"  # uniform | clustered | twocube
    charges: str = "pm1"   # pm1 (equal +1/-1, shuffled) | uniform (U[-1,1] minus mean) | biased
    seed: int = 0
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "uniform-1k-n8": Workload("uniform-1k-n8", 1000, 8, charges="pm1", seed=1001),
    "uniform-100k-n32": Workload("uniform-100k-n32", 100_000, 32, charges="uniform", seed=1002),
    "uniform-1M-n64": Workload("uniform-1M-n64", 1_000_000, 64, charges="pm1", seed=1003),
    "clustered-1M-n64": Workload("clustered-1M-n64", 1_000_000, 64, kind="clustered",
                                 charges="pm1", seed=1004,
                                 extra={"clusters": 64, "sigma": 0.02, "background": 0.1}),
}


def _charges(rng, N, mode):
    if mode == "pm1":
        if N % 2:
            raise ValueError("pm1 charges need even N")
        Q = np.concatenate([np.ones(N // 2), -np.ones(N // 2)])
        return rng.permutation(Q)
    if mode == "uniform":
        Q = rng.uniform(-1.0, 1.0, N)
        Q -= Q.mean()
        return Q
    raise ValueError(mode)


def positions_uniform(rng, N, L=1.0):
    return rng.random((N, 3)) * L


def positions_clustered(rng, N, L=1.0, clusters=64, sigma=0.02, background=0.1):
    """Isotropic Gaussian clusters (centres uniform, wrapped periodically)
    plus a uniform background fraction."""
    n_bg = int(round(background * N))
    n_cl = N - n_bg
    centres = rng.random((clusters, 3)) * L
    per = np.full(clusters, n_cl // clusters)
    per[: n_cl - per.sum()] += 1
    parts = [centres[c] + sigma * L * rng.standard_normal((per[c], 3)) for c in range(clusters)]
    parts.append(rng.random((n_bg, 3)) * L)
    x = np.concatenate(parts)
    return np.mod(x, L)


def positions_twocube(rng, N, L=1.0):
    """The paper's demonstration set-up: half the charges in each of the two
    sub-cubes [0,L/2]^3 and [L/2,L]^3, the first biased 55% positive, the
    second 55% negative (Section 4)."""
    n1 = N // 2
    n2 = N - n1
    x1 = rng.random((n1, 3)) * (L / 2)
    x2 = L / 2 + rng.random((n2, 3)) * (L / 2)
    p1 = int(round(0.55 * n1))
    p2 = n2 - int(round(0.55 * n2))
    q1 = np.concatenate([np.ones(p1), -np.ones(n1 - p1)])
    q2 = np.concatenate([np.ones(p2), -np.ones(n2 - p2)])
    Q = np.concatenate([rng.permutation(q1), rng.permutation(q2)])
    x = np.concatenate([x1, x2])
    return x, Q


def make(workload: Workload | str, seed: int | None = None):
    """Return (x [N,3] float64, Q [N] float64) for a workload."""
    w = WORKLOADS[workload] if isinstance(workload, str) else workload
    rng = np.random.Generator(np.random.PCG64(w.seed if seed is None else seed))
    if w.kind == "uniform":
        x = positions_uniform(rng, w.N, w.L)
        Q = _charges(rng, w.N, w.charges)
    elif w.kind == "clustered":
        x = positions_clustered(rng, w.N, w.L, **w.extra)
        Q = _charges(rng, w.N, w.charges)
    elif w.kind == "twocube":
        x, Q = positions_twocube(rng, w.N, w.L)
    else:
        raise ValueError(w.kind)
    return np.ascontiguousarray(x, dtype=np.float64), np.ascontiguousarray(Q, dtype=np.float64)


def uniform(N, L=1.0, seed=0, charges="pm1"):
    """Small ad-hoc uniform case (tests)."""
    return make(Workload(f"adhoc-{N}", N, 8, L=L, charges=charges, seed=seed))


def batch(B=64, n=16, Nmin=2000, Nmax=64000, seed=1005, L=1.0):
    """B independent uniform configurations with N log-uniform in [Nmin, Nmax]
    and charges U[-1,1] shifted to zero mean.  Returns lists (xs, Qs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ns = np.round(np.exp(rng.uniform(np.log(Nmin), np.log(Nmax), B))).astype(np.int64)
    xs, Qs = [], []
    for Nb in Ns:
        xs.append(positions_uniform(rng, int(Nb), L))
        Qs.append(_charges(rng, int(Nb), "uniform"))
    return xs, Qs
