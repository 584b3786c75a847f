"""CPU oracle of the batched Ising Metropolis sweep: TEST INFRASTRUCTURE ONLY.

The paper's first benchmark (main text eq. (1) and the supplement's section I.1) is the
square-lattice Ising model H = -J sum_<ij> s_i s_j, s = +-1, periodic L x L, sampled by local
Metropolis updates at T_c; a sweep attempts every spin once (supplement section I.3).  Its
printed results (Table 1) are |M| = (1/N)|sum s| and E = <H>/N.

Readings where the paper is silent:
* site order: checkerboard, all sites with (x + y) even first, then the odd ones.  Sites of one
  colour do not interact, so a colour is updated as one step, equal to any sequential order of
  its sites; the sweep is still one attempt per spin.
* acceptance: accept iff u < min(1, exp(-dE / T)), strict, u uniform in [0, 1).
* random numbers: Philox4x64-10, key (seed, 0), counter (b, 0, global sweep, 2) for the 4 sites
  4b .. 4b+3 of the row-major lattice (word q for site 4b + q), u = top 53 bits / 2^53.
* initial spins drawn like the DQMC fields: site e is +1 iff the low bit of raw word e of the
  counter blocks (e / 4, 0, 0, 0) under key (seed, 0) is 1.

Exact reference: Kaufman's partition function of the finite periodic lattice (B. Kaufman,
Phys. Rev. 76, 1232 (1949), in the four-product form), which gives the exact energy per site at
any L; pinned in the tests against enumeration of all 2^16 states of the 4 x 4 lattice.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from .philox import philox4x64_10, to_unit

STREAM_ISING = 2   # counter word 3 of the Ising acceptance stream


def bond_sum(s: np.ndarray) -> int:
    """B = sum_i s_i (s_{x+1,y} + s_{x,y+1}) on the periodic lattice s[y][x]; H = -J B."""
    s = np.asarray(s, dtype=np.int64)
    return int(np.sum(s * np.roll(s, -1, axis=1)) + np.sum(s * np.roll(s, -1, axis=0)))


def accept_prob(dE: float, T: float) -> float:
    """Metropolis acceptance min(1, exp(-dE/T))."""
    return 1.0 if dE <= 0 else math.exp(-dE / T)


def sweep_uniforms(seed: int, sweep: int, n_sites: int) -> List[float]:
    """Acceptance uniforms of one sweep, one per row-major site."""
    out = []
    for b in range((n_sites + 3) // 4):
        w = philox4x64_10((b, 0, sweep, STREAM_ISING), (seed, 0))
        out.extend(to_unit(x) for x in w)
    return out[:n_sites]


def initial_spins(seed: int, n_sites: int) -> np.ndarray:
    out = np.empty(n_sites, dtype=np.int8)
    for e in range(n_sites):
        w = philox4x64_10((e // 4, 0, 0, 0), (seed, 0))[e % 4]
        out[e] = 1 if (w & 1) else -1
    return out


class IsingChains:
    """Independent Metropolis chains of the L x L Ising model, spins[c][y*L + x]."""

    def __init__(self, L: int, J: float, T: float, spins: Optional[np.ndarray], seeds):
        self.L, self.J, self.T = L, J, T
        self.seeds = [int(s) for s in seeds]
        n = len(self.seeds)
        if spins is None:
            spins = np.stack([initial_spins(s, L * L) for s in self.seeds])
        self.s = np.array(spins, dtype=np.int8).reshape(n, L, L).copy()
        self.sweeps_done = [0] * n
        self.accepted = [0] * n
        self.n_meas = [0] * n
        self.sum_abs_m = [0] * n
        self.sum_m2 = [0] * n
        self.sum_b = [0] * n
        self.sum_b2 = [0] * n

    def sweep(self, n_sweeps: int, measure: bool = True):
        """n_sweeps sweeps of every chain; returns the series [c][sweep] of (M, B) after each."""
        L, J, T = self.L, self.J, self.T
        series = np.zeros((len(self.seeds), n_sweeps, 2), dtype=np.int64)
        for c, seed in enumerate(self.seeds):
            s = self.s[c]
            for k in range(n_sweeps):
                u = sweep_uniforms(seed, self.sweeps_done[c], L * L)
                for colour in (0, 1):
                    for y in range(L):
                        for x in range(L):
                            if (x + y) % 2 != colour:
                                continue
                            h = (int(s[y, (x + 1) % L]) + int(s[y, (x - 1) % L])
                                 + int(s[(y + 1) % L, x]) + int(s[(y - 1) % L, x]))
                            dE = 2.0 * J * int(s[y, x]) * h
                            if u[y * L + x] < accept_prob(dE, T):
                                s[y, x] = -s[y, x]
                                self.accepted[c] += 1
                self.sweeps_done[c] += 1
                m = int(np.sum(s, dtype=np.int64))
                b = bond_sum(s)
                series[c, k] = (m, b)
                if measure:
                    self.n_meas[c] += 1
                    self.sum_abs_m[c] += abs(m)
                    self.sum_m2[c] += m * m
                    self.sum_b[c] += b
                    self.sum_b2[c] += b * b
        return series

    def spins(self) -> np.ndarray:
        return self.s.reshape(len(self.seeds), -1).copy()


# ------------------------------------------------------------------------- exact results
def kaufman_log_z(L: int, K, mp=None):
    """ln Z of the L x L periodic Ising model at coupling K = J/T (Kaufman 1949):
        Z = 1/2 (2 sinh 2K)^(L^2/2) (Z1 + Z2 + Z3 + Z4),
        Z1 = prod_r 2 cosh(L g_{2r+1}/2), Z2 = prod_r 2 sinh(L g_{2r+1}/2),
        Z3 = prod_r 2 cosh(L g_{2r}/2),   Z4 = prod_r 2 sinh(L g_{2r}/2),   r = 0 .. L-1,
    with cosh g_k = cosh 2K coth 2K - cos(pi k / L) (g_k > 0) for k != 0, and
    g_0 = 2K + ln tanh K (negative above T_c, which flips the sign of Z4).
    Evaluated with mpmath at the context's precision when mp is given."""
    import mpmath
    m = mp or mpmath.mp
    K = m.mpf(K)
    c2 = m.cosh(2 * K) / m.tanh(2 * K)

    def g(k):
        if k == 0:
            return 2 * K + m.log(m.tanh(K))
        return m.acosh(c2 - m.cos(m.pi * k / L))

    z = [m.mpf(1)] * 4
    for r in range(L):
        go, ge = g(2 * r + 1), g(2 * r)
        z[0] *= 2 * m.cosh(L * go / 2)
        z[1] *= 2 * m.sinh(L * go / 2)
        z[2] *= 2 * m.cosh(L * ge / 2)
        z[3] *= 2 * m.sinh(L * ge / 2)
    return m.log(m.mpf(1) / 2) + (m.mpf(L * L) / 2) * m.log(2 * m.sinh(2 * K)) + m.log(sum(z))


def kaufman_energy(L: int, J: float, T: float) -> float:
    """Exact <H>/N = -(J/N) d ln Z / dK at K = J/T (derivative by mpmath at 50 digits)."""
    import mpmath
    with mpmath.workdps(50):
        K = mpmath.mpf(J) / mpmath.mpf(T)
        d = mpmath.diff(lambda k: kaufman_log_z(L, k), K)
        return float(-J * d / (L * L))
