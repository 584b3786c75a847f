"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module builds only *inputs*: hopping matrices of the lattices the paper's Hubbard model is
posed on, seeded +-1 Hubbard-Stratonovich (HS) fields, and the workload definitions.  It holds none
of the method's arithmetic (no propagators, no Green's functions, no update rule), so that the CPU
oracle and the HIP path can both consume it without sharing any code of the method.

Lattices (model of SM section I.1, Hamiltonian eq. (3)):
  * square, periodic boundaries, site index i = x + L*y, bonds +x and +y of every site;
  * honeycomb, periodic boundaries, 2 sites per unit cell, i = 2*(x + L*y) + sub, bonds
    A(x,y)-B(x,y), A(x,y)-B(x-1,y), A(x,y)-B(x,y-1).
Every bond adds -t to T_ij and T_ji (accumulated, so a 2-site ring gets -2t: the dispersion of a
periodic chain of length 2 is -2t cos k, which this reproduces).

Seeded fields: the paper starts its short chains from i.i.d. configurations whose elements are +1
or -1 with probability 1/2 (random inputs of the main text, and the Bernoulli discretisation of the
generated numbers in the NIMC section).  Here the random bits come from numpy's Philox4x64-10
bit generator with key (seed, 0): element e = l*N + i of the [L_tau][N] field is +1 iff the low bit
of the e-th raw 64-bit output (counter blocks 0, 1, 2, ...; four words per block) is 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


# ---------------------------------------------------------------------------- lattices
def square_hopping(L: int, t: float = 1.0) -> np.ndarray:
    """N x N hopping matrix of an L x L periodic square lattice (i = x + L*y)."""
    n = L * L
    T = np.zeros((n, n), dtype=np.float64)
    for y in range(L):
        for x in range(L):
            i = x + L * y
            for (dx, dy) in ((1, 0), (0, 1)):
                j = (x + dx) % L + L * ((y + dy) % L)
                T[i, j] += -t
                T[j, i] += -t
    return T


def honeycomb_hopping(L: int, t: float = 1.0) -> np.ndarray:
    """N x N hopping matrix of an L x L periodic honeycomb lattice, N = 2 L^2."""
    n = 2 * L * L
    T = np.zeros((n, n), dtype=np.float64)
    for y in range(L):
        for x in range(L):
            a = 2 * (x + L * y)
            for (bx, by) in ((x, y), ((x - 1) % L, y), (x, (y - 1) % L)):
                b = 2 * (bx + L * by) + 1
                T[a, b] += -t
                T[b, a] += -t
    return T


def staggered_sign(lattice: str, L: int) -> np.ndarray:
    """Diagonal of the sublattice sign D with D T D = -T (bipartite lattices)."""
    if lattice == "square":
        if L % 2:
            raise ValueError("square lattice is bipartite only for even L")
        return np.array([(-1.0) ** ((i % L) + (i // L)) for i in range(L * L)])
    if lattice == "honeycomb":
        return np.array([1.0 if i % 2 == 0 else -1.0 for i in range(2 * L * L)])
    raise ValueError(lattice)


def hopping(lattice: str, L: int, t: float = 1.0) -> np.ndarray:
    if lattice == "square":
        return square_hopping(L, t)
    if lattice == "honeycomb":
        return honeycomb_hopping(L, t)
    raise ValueError(lattice)


# ---------------------------------------------------------------------------- fields
def _philox_words(seed: int, n_words: int) -> np.ndarray:
    """First n_words raw outputs of Philox4x64-10, key (seed, 0), counter blocks 0, 1, ..."""
    # numpy increments the 256-bit counter before producing a block, so start one below 0.
    start = (1 << 256) - 1
    ctr = [(start >> (64 * w)) & ((1 << 64) - 1) for w in range(4)]
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64),
                          key=np.array([seed & ((1 << 64) - 1), 0], dtype=np.uint64))
    return bg.random_raw(n_words)


def seeded_field(seed: int, n_slices: int, n_sites: int) -> np.ndarray:
    """One chain's +-1 HS field, int8 [n_slices][n_sites]."""
    bits = _philox_words(seed, n_slices * n_sites) & np.uint64(1)
    return (2 * bits.astype(np.int8) - 1).reshape(n_slices, n_sites)


def seeded_fields(seeds, n_slices: int, n_sites: int) -> np.ndarray:
    """[n_chains][n_slices][n_sites] int8 fields, one seed per chain."""
    return np.stack([seeded_field(int(s), n_slices, n_sites) for s in seeds])


def chain_seeds(config_id: int, n_chains: int, first: int = 0) -> np.ndarray:
    """Seeds (config_id << 32) | chain for chains first .. first+n_chains-1."""
    return np.array([(config_id << 32) | (first + c) for c in range(n_chains)], dtype=np.uint64)


# ---------------------------------------------------------------------------- workloads
@dataclass
class Workload:
    """One DQMC workload: lattice, couplings, Trotter grid and chain count."""
    name: str
    config_id: int
    lattice: str
    L: int
    U: float
    beta: float
    dtau: float
    n_chains: int
    n_sweeps: int
    stab_every: int
    t: float = 1.0
    mu: float = 0.0
    precision: str = "fp64"
    refresh_every: int = 0
    delay_ranks: List[int] = field(default_factory=list)

    @property
    def n_sites(self) -> int:
        return self.L * self.L * (2 if self.lattice == "honeycomb" else 1)

    @property
    def n_slices(self) -> int:
        return int(round(self.beta / self.dtau))

    def hopping(self) -> np.ndarray:
        return hopping(self.lattice, self.L, self.t)

    def seeds(self, n: Optional[int] = None, first: int = 0) -> np.ndarray:
        return chain_seeds(self.config_id, self.n_chains if n is None else n, first)

    def fields(self, n: Optional[int] = None, first: int = 0) -> np.ndarray:
        return seeded_fields(self.seeds(n, first), self.n_slices, self.n_sites)

    @property
    def updates_per_run(self) -> int:
        return self.n_chains * self.n_sweeps * self.n_slices * self.n_sites


WORKLOADS = {
    # one chain, 4x4 square, U=4, beta=2: the small case the oracle finishes in seconds
    "square4x4_U4_b2": Workload("square4x4_U4_b2", 1, "square", 4, 4.0, 2.0, 0.1, 1, 100, 10),
    # 256 chains, 8x8 square, U=4, beta=4: the throughput workload
    "square8x8_U4_b4": Workload("square8x8_U4_b4", 2, "square", 8, 4.0, 4.0, 0.1, 256, 50, 10,
                                delay_ranks=[4, 8, 16, 32]),
    # mixed batch: honeycomb 6x6 (N=72) and 12x12 (N=288), U=3, beta=6, FP32 wraps
    "honeycomb6x6_U3_b6": Workload("honeycomb6x6_U3_b6", 3, "honeycomb", 6, 3.0, 6.0, 0.1, 256, 15,
                                   10, precision="fp32_wrap", refresh_every=10),
    "honeycomb12x12_U3_b6": Workload("honeycomb12x12_U3_b6", 3, "honeycomb", 12, 3.0, 6.0, 0.1,
                                     256, 15, 10, precision="fp32_wrap", refresh_every=10),
    # large-N stress: 20x20 square, U=8, beta=10
    "square20x20_U8_b10": Workload("square20x20_U8_b10", 5, "square", 20, 8.0, 10.0, 0.1, 64, 15,
                                   10, delay_ranks=[16, 32, 64]),
    # the paper's honeycomb point (L=6, U=3.83, beta=6, dtau=0.1; 15 sweeps from 1000 chains)
    "honeycomb6x6_U3.83_b6": Workload("honeycomb6x6_U3.83_b6", 6, "honeycomb", 6, 3.83, 6.0, 0.1,
                                      1000, 15, 10),
}

# serving stream: square lattice, t=1, U=4, dtau=0.1, L in {4,...,16}, beta in {2,4,8}
SERVING_L = (4, 6, 8, 10, 12, 16)
SERVING_BETA = (2.0, 4.0, 8.0)
SERVING_SWEEPS = (20, 200)
SERVING_RATES = (50, 100, 200, 500, 1000, 2000)


def serving_requests(n: int, rate: float, seed: int = 4, Ls=SERVING_L):
    """Poisson arrivals at `rate` req/s with L (from `Ls`), beta and sweep count drawn uniformly;
    seeded.  Restricting `Ls` keeps the arrival rate: the stream is drawn over the given lattices."""
    rng = np.random.Generator(np.random.Philox(key=[seed, int(rate)]))
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps)
    reqs = []
    for r in range(n):
        L = int(rng.choice(Ls))
        beta = float(rng.choice(SERVING_BETA))
        sweeps = int(rng.integers(SERVING_SWEEPS[0], SERVING_SWEEPS[1] + 1))
        reqs.append(dict(id=r, arrival=float(arrivals[r]), L=L, beta=beta, sweeps=sweeps,
                         seed=(4 << 32) | r))
    return reqs
