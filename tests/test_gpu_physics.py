"""Markov-chain statistics of the HIP path against exact results.

The 2x2 square lattice has a 256-dimensional Fock space, so the Trotterised model of eq. (3) is
traced exactly (tests/exact_tools.py) at any L_tau; the discrete HS transformation reproduces that
trace term by term, so chains that sample W(s) correctly must reproduce its double occupancy,
kinetic energy and staggered structure factor within their statistical errors (mean over
independent chains of each chain's time average; 4 sigma).
"""
import math

import numpy as np
import pytest

import dqmc_inputs as di
import exact_tools as ex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_00712_amd import dqmc
    dqmc.lib()
    return dqmc


@pytest.mark.parametrize("precision,refresh", [("fp64", 0), ("fp32_wrap", 5)])
def test_chain_statistics_match_fock_trace_2x2(dq, precision, refresh):
    T = di.square_hopping(2)
    U, dtau, Lt = 4.0, 0.1, 20
    eps = di.staggered_sign("square", 2)
    _, d_x, e_x, s_x = ex.fock_trotter(T, U, dtau, Lt, form=eps)
    n_chains, burn, n_meas = 256, 30, 200
    m = dq.make_model(T, U, dtau, Lt, 5, refresh_every=refresh, precision=precision)
    b = dq.Batch(m, di.chain_seeds(9, n_chains))
    b.sweep(burn)
    sums = np.zeros((n_chains, 3))
    for _ in range(n_meas):
        b.sweep(1)
        o = b.measure()
        s = b.spin_structure(eps).cpu().numpy()
        sums += np.stack([o["double_occ"], o["kinetic"], s], axis=1)
    assert not np.any(o["flags"])
    means = sums / n_meas
    for k, exact in enumerate((d_x, e_x, s_x)):
        mu = means[:, k].mean()
        se = means[:, k].std(ddof=1) / math.sqrt(n_chains)
        assert abs(mu - exact) < 4 * se, (k, mu, se, exact)
