"""Seeded request trace for the serving workload (input data only).

Requests arrive as a Poisson process (mean rate `rate` per second, seed
`seed`).  Request j draws from its own generator (seed 1000 + j): the
lattice (square NN t=-1 with NNN t'=0.1, or graphene t=-2.7, each with
probability 1/2), the orbital count log-uniform on [n_min, n_max] (square:
L = round(sqrt(n)); graphene: L = round(sqrt(n / 2))), the number of random
vectors uniform on 1..r_max, the number of time steps uniform on `steps`,
and FP32 or FP64 with probability 1/2.  All lattices are clean and periodic.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np


@dataclass
class TraceRequest:
    index: int
    arrival: float          # seconds after the trace starts
    lattice: str            # "square_nnn" or "graphene"
    dims: int               # L (L x L cells)
    vectors: int
    time_steps: int
    fp32: bool
    seed: int

    @property
    def rescale(self) -> float:
        return 4.5 if self.lattice == "square_nnn" else 9.0

    @property
    def orbitals(self) -> int:
        return self.dims * self.dims * (1 if self.lattice == "square_nnn" else 2)


def serving_trace(num_requests: int = 64, rate: float = 50.0, seed: int = 4, n_min: float = 1e4,
                  n_max: float = 1e7, r_max: int = 32,
                  steps: Sequence[int] = (128, 256, 512, 1024, 2048)) -> List[TraceRequest]:
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=num_requests))
    out = []
    for j in range(num_requests):
        g = np.random.default_rng(1000 + j)
        lattice = "square_nnn" if g.random() < 0.5 else "graphene"
        n = float(np.exp(g.uniform(np.log(n_min), np.log(n_max))))
        dims = int(round(np.sqrt(n if lattice == "square_nnn" else n / 2)))
        dims = max(dims, 4)
        vectors = int(g.integers(1, r_max + 1))
        nt = int(g.choice(np.asarray(steps)))
        fp32 = bool(g.random() < 0.5)
        out.append(TraceRequest(j, float(arrivals[j]), lattice, dims, vectors, nt, fp32, 1000 + j))
    return out


def build_lattice(req: TraceRequest):
    from .lattices import graphene, square
    if req.lattice == "square_nnn":
        return square(req.dims)
    return graphene(req.dims)
