"""Philox4x64-10 counter-based generator, oracle side (test infrastructure only).

Written from the published definition (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 64x64->128-bit
multiplications on a 4-word counter with a 2-word key bumped by Weyl constants between rounds.

The paper states no random-number generator; the acceptance uniforms of the DQMC sweep are drawn
from this generator so that every chain's trajectory is a pure function of its seed and its
global sweep counter (independent of batching).  Pinned bit-for-bit against numpy.random.Philox.
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B

STREAM_FIELD = 0      # counter word 3 of the initial-field stream (kept for documentation)
STREAM_ACCEPT = 1     # counter word 3 of the acceptance-uniform stream


def philox4x64_10(ctr, key):
    """Return the four 64-bit output words for counter ctr[0..3] and key key[0..1]."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & MASK64
            k1 = (k1 + _W1) & MASK64
        p0 = _M0 * x0
        p1 = _M1 * x2
        x0, x1, x2, x3 = ((p1 >> 64) ^ x1 ^ k0, p1 & MASK64, (p0 >> 64) ^ x3 ^ k1, p0 & MASK64)
    return x0, x1, x2, x3


def to_unit(x: int) -> float:
    """Top 53 bits of a 64-bit word as a double in [0, 1)."""
    return (int(x) >> 11) * (1.0 / 9007199254740992.0)


def accept_uniform(seed: int, sweep: int, slice_idx: int, site: int) -> float:
    """Uniform for the attempt at (global sweep, 0-based slice, site) of the chain with this seed."""
    w = philox4x64_10((site, slice_idx, sweep, STREAM_ACCEPT), (seed, 0))
    return to_unit(w[0])
