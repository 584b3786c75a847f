"""GPU parity of the sweep modes (dqmc_model.sweep_mode): alternating up/down sweeps that reuse
the UDT stacks, and per-slice equal-time estimators, against the oracle's same conventions.

Trajectories bit for bit (unless a near tie |u - R| < 1e-9 was met on either side), per-slice
averages and observables to 1e-9, as the other trajectory tests.
"""
import math

import numpy as np
import pytest

import dqmc_inputs as di
import exact_tools as ex

pytestmark = pytest.mark.gpu

SQUARE12 = di.Workload("square12x12_U4_b2", 9, "square", 12, 4.0, 2.0, 0.1, 1, 1, 10)


@pytest.fixture(scope="module")
def dq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_00712_amd import dqmc
    dqmc.lib()
    return dqmc


def _check(dq, w, n, sweeps, mode, first=0):
    from oracle import Model, OracleChains
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, sweep_mode=mode)
    b = dq.Batch(m, w.seeds(n, first), w.fields(n, first))
    assert b.variant in (0, 1)          # the workspace kernels at any N
    om = Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, sweep_mode=mode)
    oc = OracleChains(om, w.fields(n, first), w.seeds(n, first))
    b.sweep(sweeps)
    oc.sweep(sweeps)
    obs = b.measure()
    ref = oc.measure()
    f_gpu = b.fields().cpu().numpy()
    for c in range(n):
        if obs["near_ties"][c] or ref[c]["near_ties"]:
            continue
        assert np.array_equal(f_gpu[c], oc.fields()[c]), f"chain {c}"
        assert obs["accepted"][c] == ref[c]["accepted"]
        assert abs(obs["double_occ"][c] - ref[c]["double_occ"]) < 1e-9
        assert obs["slice_meas"][c] == ref[c]["slice_meas"]
        if mode & 2:
            assert abs(obs["slice_double_occ"][c] - ref[c]["slice_double_occ"]) < 1e-9
            assert abs(obs["slice_kinetic"][c] - ref[c]["slice_kinetic"]) < 1e-9
        assert obs["flags"][c] == 0 and obs["max_drift"][c] < 1e-6
    return b, obs


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_square4x4_sweep_modes(dq, mode):
    """N = 16 in the workspace kernels: three up and three down sweeps."""
    b, obs = _check(dq, di.WORKLOADS["square4x4_U4_b2"], 1, 6, mode)
    assert obs["sweeps_done"][0] == 6


def test_square8x8_alternating_with_slices(dq):
    _check(dq, di.WORKLOADS["square8x8_U4_b4"], 2, 3, 3)


def test_honeycomb6x6_alternating(dq):
    _check(dq, di.WORKLOADS["honeycomb6x6_U3_b6"], 1, 2, 1)


def test_square12x12_alternating_two_level_delay(dq):
    """N = 144: the accumulated delayed-update panels in both sweep directions."""
    b, _ = _check(dq, SQUARE12, 1, 2, 3)
    assert b.delay_rank == 32


def test_alternating_resume_and_probe(dq):
    """The direction follows the global sweep counter: 3 + 2 sweeps equal 5; a fixed-field probe
    between sweeps (which borrows the right stack as scratch) does not change the trajectory."""
    w = di.WORKLOADS["square4x4_U4_b2"]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, sweep_mode=1)
    a = dq.Batch(m, w.seeds(2), w.fields(2))
    a.sweep(5)
    b = dq.Batch(m, w.seeds(2), w.fields(2))
    b.sweep(3)
    b.debug_green(7, 0)
    b.sweep(2)
    oa, ga = a.measure(green=True)
    ob, gb = b.measure(green=True)
    assert np.array_equal(a.fields().cpu().numpy(), b.fields().cpu().numpy())
    assert np.array_equal(oa["accepted"], ob["accepted"])
    assert np.max(np.abs(ga.cpu().numpy() - gb.cpu().numpy())) < 1e-12


def test_alternating_per_slice_statistics_match_fock_trace_2x2(dq):
    """2x2, U = 4, beta = 2, alternating sweeps with per-slice estimators: chain averages of the
    per-slice double occupancy and kinetic energy within 4 sigma of the exact Trotter trace."""
    T = di.square_hopping(2)
    U, dtau, Lt = 4.0, 0.1, 20
    _, d_x, e_x = ex.fock_trotter(T, U, dtau, Lt)
    n_chains, burn, n_meas = 256, 30, 100
    m = dq.make_model(T, U, dtau, Lt, 5, sweep_mode=3)
    b = dq.Batch(m, di.chain_seeds(10, n_chains))
    b.sweep(burn)
    o0 = b.measure()
    b.sweep(n_meas)
    o1 = b.measure()
    assert not np.any(o1["flags"])
    n0, n1 = o0["slice_meas"].astype(float), o1["slice_meas"].astype(float)
    assert np.all(n1 - n0 == n_meas * Lt)
    for key, exact in (("slice_double_occ", d_x), ("slice_kinetic", e_x)):
        per = (o1[key] * n1 - o0[key] * n0) / (n1 - n0)
        mu, se = per.mean(), per.std(ddof=1) / math.sqrt(n_chains)
        assert abs(mu - exact) < 4 * se, (key, mu, se, exact)


@pytest.mark.parametrize("name,mode", [("square4x4_U4_b2", 0), ("square8x8_U4_b4", 3),
                                       ("honeycomb6x6_U3_b6", 1)])
def test_unwrap_parity(dq, name, mode):
    """Fixed fields: fresh G(l), then the down sweeps' unwraps G <- B_l^{-1} G B_l, against the
    oracle's, to 1e-10 relative (both stay within 1e-12 of the fresh G(l - k))."""
    from oracle import Model, OracleChains
    w = di.WORKLOADS[name]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, sweep_mode=mode)
    b = dq.Batch(m, w.seeds(2), w.fields(2))
    oc = OracleChains(Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every), w.fields(2), w.seeds(2))
    for sl, nw in ((w.stab_every, -1), (w.stab_every, -3), (w.n_slices, -5)):
        g = b.debug_green(sl, nw).cpu().numpy()
        ref = oc.debug_green(sl, nw)
        assert np.max(np.abs(g - ref)) / max(1.0, np.max(np.abs(ref))) < 1e-10, (sl, nw)
