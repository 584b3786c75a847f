"""FP32-wrap precision: FP32 MFMA wraps and delayed updates, FP64 stabilisation and ratios.

* The bound max|dG| <= 1e-5 is checked against the FP64 oracle on fixed fields at the refresh
  interval the autotuner picks for each workload (the interval the benchmark runs), after exactly
  that many FP32 wraps from a fresh G: the FP32-wrapped G against the oracle's fresh G of the
  same slice (supplement section I.2 defines the G being approximated).
* The drift flag fires at the bound: a chain is flagged exactly when its drift at a refresh point
  exceeded the model's drift_limit (1e-5 by default in FP32_WRAP).
* FP32-wrap chains stay sound: half filling, observables close to the FP64 run's.
"""
import numpy as np
import pytest

import dqmc_inputs as di

pytestmark = pytest.mark.gpu

BOUND = 1e-5


@pytest.fixture(scope="module")
def dq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_00712_amd import dqmc
    dqmc.lib()
    return dqmc


@pytest.mark.parametrize("name", ["square8x8_U4_b4", "square4x4_U4_b2"])
def test_fp32_wrap_error_grows_with_wraps(dq, name):
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
        ref = oc.debug_green(10 + nw, 0)
        errs[nw] = float(np.max(np.abs(g - ref)))
    print(name, errs)
    assert errs[0] < 1e-6          # the fresh G is FP64, stored as FP32: rounding only
    assert errs[2] < BOUND
    assert errs[8] >= errs[1]      # what the refresh interval controls


# The honeycomb lattices (72 and 288 sites) run FP32 wraps in the workspace kernels; a run of those
# kernels in FP32 made a GPU memory fault once (serving mix, 100 sites) with no cause found on the
# CPU, so they stay off the GPU until one is.
FP32_WS_OFF = pytest.mark.skip(reason="FP32 workspace kernels kept off the GPU after an "
                                      "unexplained memory fault")


@pytest.mark.parametrize("name,n_chains", [("square8x8_U4_b4", 4),
                                           pytest.param("honeycomb6x6_U3_b6", 2, marks=FP32_WS_OFF),
                                           pytest.param("honeycomb12x12_U3_b6", 2, marks=FP32_WS_OFF)])
def test_fp32_bound_at_the_tuned_refresh_vs_oracle(dq, name, n_chains):
    """The refresh interval r* the autotuner picks (GPU FP32 wraps against the GPU FP64 fresh G
    on fixed fields) keeps the FP32-wrapped G within 1e-5 of the oracle's fresh G after r*
    wraps, on chains and slices other than the ones it was tuned on."""
    from oracle import Model, OracleChains
    from paper_2106_00712_amd.autotune import Autotuner
    w = di.WORKLOADS[name]
    tuned = Autotuner().refresh_interval(w.hopping(), w.U, w.dtau, w.n_slices, w.fields(n_chains),
                                         w.seeds(n_chains), bound=BOUND,
                                         candidates=(2, 3, 4, 5, 6, 8, 10), stab_every=w.stab_every)
    r = tuned["refresh_every"]
    assert r >= 2
    first = 100            # chains the autotuner did not see
    f, s = w.fields(n_chains, first), w.seeds(n_chains, first)
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, precision="fp32_wrap",
                      refresh_every=r)
    b = dq.Batch(m, s, f)
    oc = OracleChains(Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every), f, s)
    worst = 0.0
    for l in sorted({0, w.n_slices // 2, w.n_slices - r}):
        g = b.debug_green(l, r).cpu().numpy()
        ref = oc.debug_green(l + r, 0)
        worst = max(worst, float(np.max(np.abs(g - ref))))
    print(name, "r* =", r, "max|dG| vs oracle =", worst, tuned["max_abs_dG"])
    assert worst <= BOUND


def test_fp32_drift_flag_fires_at_the_bound(dq):
    w = di.WORKLOADS["square8x8_U4_b4"]
    n = 32
    flagged = {}
    for limit in (0.0, 1.0):       # 0: the FP32_WRAP default, 1e-5
        m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, precision="fp32_wrap",
                          refresh_every=3, drift_limit=limit)
        b = dq.Batch(m, w.seeds(n), w.fields(n))
        b.sweep(2)
        o = b.measure()
        flagged[limit] = (o["flags"] & dq.FLAG_DRIFT) != 0
        if limit == 0.0:
            assert np.array_equal(flagged[limit], o["max_drift"] > BOUND)
            drift = o["max_drift"]
        else:
            assert not flagged[limit].any()
            assert np.array_equal(o["max_drift"], drift)    # the limit changes only the flag
    print("chains over 1e-5 after 2 sweeps:", int(flagged[0.0].sum()), "of", n,
          "max drift", float(drift.max()))


def test_fp32_chains_are_sound(dq):
    w = di.WORKLOADS["square8x8_U4_b4"]
    n = 16
    m32 = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, precision="fp32_wrap",
                        refresh_every=4, drift_limit=1e-2)
    b = dq.Batch(m32, w.seeds(n), w.fields(n))
    assert b.stab == 4
    b.sweep(3)
    obs = b.measure()
    assert np.all(obs["flags"] == 0)
    assert np.all(np.abs(obs["density"] - 1.0) < 1e-9)   # the fresh FP64 G keeps half filling
    assert float(obs["max_drift"].max()) < 1e-2
    assert np.all(obs["attempted"] == 3 * w.n_slices * w.n_sites)
    m64 = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    b64 = dq.Batch(m64, w.seeds(n), w.fields(n))
    b64.sweep(3)
    o64 = b64.measure()
    # same seeds and starting fields: ensembles after 3 sweeps agree statistically
    d32, d64 = obs["double_occ"], o64["double_occ"]
    se = np.sqrt(d32.var(ddof=1) / n + d64.var(ddof=1) / n)
    assert abs(d32.mean() - d64.mean()) < 4 * se + 1e-6
