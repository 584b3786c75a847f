"""FP32-wrap precision: FP32 MFMA wraps and delayed updates, FP64 stabilisation and ratios.

Checks max|dG| of the FP32 wraps against the FP64 oracle on fixed fields (the quantity the
refresh interval must keep below 1e-5), and that FP32-wrap chains stay sound: half filling,
no flags, FP64 refresh drift below the bound, observables close to the FP64 run's.
"""
import numpy as np
import pytest

import dqmc_inputs as di

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_00712_amd import dqmc
    dqmc.lib()
    return dqmc


@pytest.mark.parametrize("name", ["square8x8_U4_b4", "square4x4_U4_b2"])
def test_fp32_wrap_error_vs_oracle(dq, name):
    from oracle import Model, OracleChains
    w = di.WORKLOADS[name]
    n = 3
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, precision="fp32_wrap",
                      refresh_every=w.stab_every)
    b = dq.Batch(m, w.seeds(n), w.fields(n))
    oc = OracleChains(Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every), w.fields(n), w.seeds(n))
    errs = {}
    for nw in (0, 1, 2, 4, 8):
        g = b.debug_green(10, nw).cpu().numpy()
        ref = oc.debug_green(10, nw)
        errs[nw] = float(np.max(np.abs(g - ref)))
    print(name, errs)
    # the fresh G is FP64, stored as FP32: rounding only
    assert errs[0] < 1e-6
    # a few FP32 wraps stay inside the 1e-5 budget
    assert errs[2] < 1e-5
    # and the error grows with the number of wraps (what the refresh interval controls)
    assert errs[8] >= errs[1]


def test_fp32_chains_are_sound(dq):
    w = di.WORKLOADS["square8x8_U4_b4"]
    n = 16
    m32 = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, precision="fp32_wrap",
                        refresh_every=4)
    b = dq.Batch(m32, w.seeds(n), w.fields(n))
    assert b.stab == 4
    b.sweep(3)
    obs = b.measure()
    assert np.all(obs["flags"] == 0)
    assert np.all(np.abs(obs["density"] - 1.0) < 1e-9)   # the fresh FP64 G keeps half filling
    assert float(obs["max_drift"].max()) < 1e-3
    assert np.all(obs["attempted"] == 3 * w.n_slices * w.n_sites)
    m64 = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    b64 = dq.Batch(m64, w.seeds(n), w.fields(n))
    b64.sweep(3)
    o64 = b64.measure()
    # same seeds and starting fields: ensembles after 3 sweeps agree statistically
    d32, d64 = obs["double_occ"], o64["double_occ"]
    se = np.sqrt(d32.var(ddof=1) / n + d64.var(ddof=1) / n)
    assert abs(d32.mean() - d64.mean()) < 4 * se + 1e-6
