"""dqmc_run_static, the entry point for callers that cannot allocate device memory: the same
kernels as dqmc_init_chains -> dqmc_sweep -> dqmc_measure with the chains' state in the library's
static device array.  Two calls in a row, the second smaller than the first, each compared bit
for bit with the workspace path on the same inputs; and the size limit."""
import numpy as np
import pytest

import dqmc_inputs as di

pytestmark = pytest.mark.gpu

OBS_KEYS = ("double_occ", "density", "kinetic", "logdet_up", "logdet_dn", "max_drift",
            "max_logdet_err", "attempted", "accepted", "near_ties", "sweeps_done", "flags")


@pytest.fixture(scope="module")
def dq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_00712_amd import dqmc
    dqmc.lib()
    return dqmc


def _workspace_run(dq, w, n, sweeps, fields):
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    b = dq.Batch(m, w.seeds(n), fields)
    b.sweep(sweeps)
    o, g = b.measure(green=True)
    f = b.fields()
    return o, g.cpu().numpy(), f.cpu().numpy()


def test_run_static_equals_workspace_path_twice(dq):
    cases = [(di.WORKLOADS["square8x8_U4_b4"], 16, 2, True),    # first call: 8x8, 16 chains
             (di.WORKLOADS["square4x4_U4_b2"], 3, 3, False)]    # second: smaller, fields from seeds
    for w, n, sweeps, given in cases:
        fields = w.fields(n) if given else None
        m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
        o, g, f = dq.run_static(m, w.seeds(n), fields, n_sweeps=sweeps, green=True)
        ro, rg, rf = _workspace_run(dq, w, n, sweeps, fields)
        for k in OBS_KEYS:
            assert np.array_equal(o[k], ro[k]), (w.name, k)
        assert np.array_equal(g.cpu().numpy(), rg)
        assert np.array_equal(f.cpu().numpy(), rf)
        assert np.all(o["sweeps_done"] == sweeps)


def test_run_static_rejects_what_does_not_fit(dq):
    w = di.WORKLOADS["square8x8_U4_b4"]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    too_many = dq.STATIC_BYTES // dq.chain_bytes(m) + 1
    with pytest.raises(dq.DqmcError) as e:
        dq.run_static(m, w.seeds(too_many), None, n_sweeps=1)
    assert e.value.status == -1 and "static array" in str(e.value)
    # the array is still usable after the refusal
    o, _, _ = dq.run_static(m, w.seeds(2), w.fields(2), n_sweeps=1)
    assert np.all(o["sweeps_done"] == 1)
