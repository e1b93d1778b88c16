"""Seeded synthetic workloads: the graph parameters every run draws from.

This module describes inputs only -- scales, edge factor, Kronecker
initiator, seeds, and the scale mix of the many-small-graphs batch.  It
holds none of the pipeline's arithmetic (the generator itself is kernel K0)
and is shared by the tests and the benchmark so that the GPU library and
the CPU oracle are fed identical parameters.

Workload shapes follow the paper's benchmark definition (Sec. IV.A: N = 2^S
vertices, M = k*N edges with k = 16, Graph500 Kronecker initiator) at the
scales used here: 10 and 20 (FP64 parity), 22 (32 right-hand sides),
24 (FP32 vs FP64), 26 (largest single-GPU instance) and a batch of 512
graphs with scales drawn uniformly from 8..14.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

BASE_SEED = 1603
EDGE_FACTOR = 16
INITIATOR = (0.57, 0.19, 0.19, 0.05)
DAMPING = 0.85
ITERATIONS = 20


@dataclass(frozen=True)
class GraphSpec:
    scale: int
    edge_factor: int = EDGE_FACTOR
    a: float = INITIATOR[0]
    b: float = INITIATOR[1]
    c: float = INITIATOR[2]
    d: float = INITIATOR[3]
    seed: int = BASE_SEED

    @property
    def n(self) -> int:
        return 1 << self.scale

    @property
    def m(self) -> int:
        return self.edge_factor << self.scale

    def with_seed(self, seed: int) -> "GraphSpec":
        return replace(self, seed=seed)

    def as_dict(self) -> dict:
        return dict(scale=self.scale, edge_factor=self.edge_factor, a=self.a, b=self.b,
                    c=self.c, d=self.d, seed=self.seed)


def pipeline(scale: int, seed: int = BASE_SEED) -> GraphSpec:
    return GraphSpec(scale=scale, seed=seed)


def batch(count: int = 512, lo: int = 8, hi: int = 14, seed: int = BASE_SEED) -> list[GraphSpec]:
    """`count` independent graphs, scale uniform on [lo, hi], own seeds."""
    rng = np.random.default_rng(seed)
    scales = rng.integers(lo, hi + 1, size=count)
    seeds = rng.integers(1, 2**62, size=count, dtype=np.int64)
    return [GraphSpec(scale=int(s), seed=int(z)) for s, z in zip(scales, seeds)]


# Named workloads: the FP64 parity cases, the precision form, the two
# batching forms and the largest single-GPU instance.
WORKLOADS = {
    "kron-s10-f64": dict(scale=10, dtype="f64", nrhs=1),
    "kron-s20-f64": dict(scale=20, dtype="f64", nrhs=1),
    "kron-s24-f32": dict(scale=24, dtype="f32", nrhs=1),
    "kron-s22-f32-rhs32": dict(scale=22, dtype="f32", nrhs=32),
    "kron-batch512-s8to14-f32": dict(scale=None, dtype="f32", nrhs=1, graphs=512),
    "kron-s26-f32": dict(scale=26, dtype="f32", nrhs=1),
}
