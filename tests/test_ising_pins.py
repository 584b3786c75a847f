"""Pins of the Ising oracle (oracle/ising_oracle.py) against what fixes the values independently:
enumeration of all states, Kaufman's exact finite-lattice solution, the T -> infinity and T -> 0
limits of the Metropolis rule, and the shared seeded-input rule."""
import math

import numpy as np
import pytest

import dqmc_inputs as di
from oracle.ising_oracle import (IsingChains, bond_sum, initial_spins, kaufman_energy,
                                 kaufman_log_z, sweep_uniforms)
from oracle import philox4x64_10, to_unit


def _enumerate(L, T, J=1.0):
    """Exact ln Z, <E>/N, <|M|>/N, <M^2>/N^2 by summing over all 2^(L*L) states."""
    n = L * L
    idx = np.arange(1 << n, dtype=np.int64)
    S = np.where(((idx[:, None] >> np.arange(n)) & 1) == 1, 1, -1).reshape(-1, L, L)
    B = np.zeros(len(S), dtype=np.int64)
    for y in range(L):               # every bond once: right and down neighbour of each site
        for x in range(L):
            B += S[:, y, x] * (S[:, y, (x + 1) % L] + S[:, (y + 1) % L, x])
    M = S.reshape(len(S), -1).sum(1)
    a = J * B / T
    w = np.exp(a - a.max())
    Z = w.sum()
    return (float(np.log(Z) + a.max()), float(-J * (w * B).sum() / Z / n),
            float((w * np.abs(M)).sum() / Z / n), float((w * M * M).sum() / Z / n / n))


@pytest.mark.parametrize("L", [2, 4])
@pytest.mark.parametrize("T", [1.2, 2.269, 4.0])
def test_kaufman_equals_enumeration(L, T):
    lnz, e, _, _ = _enumerate(L, T)
    assert math.isclose(float(kaufman_log_z(L, 1.0 / T)), lnz, rel_tol=1e-13)
    assert math.isclose(kaufman_energy(L, 1.0, T), e, rel_tol=1e-11)


def test_kaufman_approaches_onsager():
    """At T_c = 2/ln(1 + sqrt 2) the energy per site tends to Onsager's -sqrt(2) with a 1/L
    correction (the specific-heat exponent is 0): L (E_L + sqrt 2) settles to a constant."""
    tc = 2.0 / math.log(1.0 + math.sqrt(2.0))
    scaled = [L * (kaufman_energy(L, 1.0, tc) + math.sqrt(2.0)) for L in (64, 128, 256)]
    assert max(scaled) - min(scaled) < 1e-2 * abs(scaled[2])
    assert abs(scaled[2] / 256) < 3e-3


def test_bond_sum_counts_each_bond_once():
    rng = np.random.default_rng(3)
    for L in (3, 4, 7):
        s = rng.choice([-1, 1], size=(L, L))
        bonds = set()
        for y in range(L):
            for x in range(L):
                bonds.add(((y, x), (y, (x + 1) % L)))
                bonds.add(((y, x), ((y + 1) % L, x)))
        assert bond_sum(s) == sum(int(s[a]) * int(s[b]) for a, b in bonds)


def test_uniforms_and_initial_spins_follow_philox():
    seed = (6 << 32) | 11
    u = sweep_uniforms(seed, 5, 10)
    for site in range(10):
        w = philox4x64_10((site // 4, 0, 5, 2), (seed, 0))[site % 4]
        assert u[site] == to_unit(w)
    assert np.array_equal(initial_spins(seed, 36), di.seeded_field(seed, 1, 36)[0])


def test_infinite_temperature_flips_every_spin():
    """T -> infinity: every proposal is accepted, so each sweep negates the lattice."""
    ch = IsingChains(4, 1.0, 1e300, None, [1, 2])
    s0 = ch.spins()
    ch.sweep(1)
    assert np.array_equal(ch.spins(), -s0) and ch.accepted == [16, 16]
    ch.sweep(1)
    assert np.array_equal(ch.spins(), s0)


def test_zero_temperature_never_raises_energy():
    """T -> 0: only moves with dE <= 0 pass, so the energy never increases; the ordered state
    is absorbing."""
    ch = IsingChains(6, 1.0, 1e-3, None, [7, 8, 9])
    ser = ch.sweep(6)
    assert np.all(np.diff(-ser[:, :, 1], axis=1) <= 0)
    up = IsingChains(4, 1.0, 1e-3, np.ones((1, 16)), [4])
    up.sweep(3)
    assert up.accepted == [0] and np.all(up.spins() == 1)


def test_measurement_sums_match_series():
    ch = IsingChains(4, 1.0, 2.269, None, [21, 22])
    ser = ch.sweep(5)
    for c in range(2):
        assert ch.sum_abs_m[c] == int(np.abs(ser[c, :, 0]).sum())
        assert ch.sum_b2[c] == int((ser[c, :, 1] ** 2).sum())
        assert ser[c, -1, 1] == bond_sum(ch.spins()[c].reshape(4, 4))


@pytest.mark.slow
def test_chain_statistics_match_enumeration_4x4():
    """Oracle chains at T = 2.269 sample the Boltzmann weight: <|M|>, <E> and <M^2> of the 4x4
    lattice within 4 sigma of exact enumeration (mean over independent chains)."""
    T = 2.269
    _, e_x, am_x, m2_x = _enumerate(4, T)
    n_chains, burn, n_meas = 24, 50, 500
    ch = IsingChains(4, 1.0, T, None, range(500, 500 + n_chains))
    ch.sweep(burn, measure=False)
    ser = ch.sweep(n_meas).astype(np.float64)
    per = np.stack([np.abs(ser[:, :, 0]).mean(1) / 16, -ser[:, :, 1].mean(1) / 16,
                    (ser[:, :, 0] ** 2).mean(1) / 256], axis=1)
    for k, exact in enumerate((am_x, e_x, m2_x)):
        mu, se = per[:, k].mean(), per[:, k].std(ddof=1) / math.sqrt(n_chains)
        assert abs(mu - exact) < 4 * se, (k, mu, se, exact)
