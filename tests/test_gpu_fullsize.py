"""Parity at the workloads' full sizes, in the launch configurations that bench.py times: sampled
chains against the oracle one by one, and every chain against identities that hold at any size.

At mu = 0 on a bipartite lattice (supplement section I.2 with the sublattice sign D, D T D = -T)
every field satisfies G_dn = D (I - G_up^T) D, hence n_up + n_dn = 1 on each site, and
log det(I + B_dn) = log det(I + B_up) - nu sum_{l,i} s_{l,i}.  The GPU computes the two spins
independently, so these tie its two Green's functions together for every chain of the batch.
"""
import math

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


def _nu(U, dtau):
    return math.acosh(math.exp(0.5 * U * dtau))


def _check_identities(w, g, obs, fields, tol_g=1e-9):
    """g: [c][2][N][N] numpy, obs: per-chain observables, fields: [c][L][N] int8."""
    D = di.staggered_sign(w.lattice, w.L)
    N = w.n_sites
    I = np.eye(N)
    nu = _nu(w.U, w.dtau)
    for c in range(g.shape[0]):
        gu, gd = g[c, 0], g[c, 1]
        assert np.all(np.isfinite(gu)) and np.all(np.isfinite(gd)), c
        assert np.max(np.abs(gd - D[:, None] * (I - gu.T) * D[None, :])) < tol_g, c
        ld = obs["logdet_up"][c] - nu * float(fields[c].astype(np.int64).sum())
        assert abs(obs["logdet_dn"][c] - ld) < 1e-8 * max(1.0, abs(ld)), c
    assert np.allclose(obs["density"], 1.0, atol=1e-9)
    assert not np.any(obs["flags"])


def test_square8x8_256_chains(dq):
    """The throughput workload as bench.py launches it (256 chains, one sweep per launch):
    three sampled chains bit for bit against the oracle after two sweeps, every chain through
    the identities."""
    from oracle import Model, OracleChains
    w = di.WORKLOADS["square8x8_U4_b4"]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    seeds, fields = w.seeds(), w.fields()
    b = dq.Batch(m, seeds, fields)
    assert b.n_chains == 256 and b.variant == 2
    b.sweep(1)
    b.sweep(1)
    obs, g = b.measure(green=True)
    f_gpu = b.fields().cpu().numpy()
    _check_identities(w, g.cpu().numpy(), obs, f_gpu)
    om = Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    for c in (0, 137, 255):
        oc = OracleChains(om, fields[c:c + 1], seeds[c:c + 1])
        oc.sweep(2)
        ref = oc.measure()[0]
        if obs["near_ties"][c] or ref["near_ties"]:
            continue
        assert np.array_equal(f_gpu[c], oc.fields()[0]), c
        assert obs["accepted"][c] == ref["accepted"]
        assert abs(obs["double_occ"][c] - ref["double_occ"]) < 1e-9
        assert abs(obs["kinetic"][c] - ref["kinetic"]) < 1e-9


def _ph_residual(g, D):
    """max |G_dn - D (I - G_up^T) D| relative to max(1, max |G|), for one chain's [2][N][N]."""
    I = np.eye(g.shape[-1])
    r = np.max(np.abs(g[1] - D[:, None] * (I - g[0].T) * D[None, :]))
    return float(r / max(1.0, float(np.max(np.abs(g)))))


@pytest.mark.parametrize("name,slice_,n_chains,sample,qr_blocked", [
    ("honeycomb6x6_U3_b6", 30, 256, (5, 200), True),
    ("honeycomb12x12_U3_b6", 30, 256, (77,), True),
    ("square20x20_U8_b10", 50, 64, (41,), False),
])
def test_fixed_field_green_full_batch(dq, name, slice_, n_chains, sample, qr_blocked):
    """The mixed-size and large-lattice workloads at their chain counts (QR as the autotuner picks
    it for each model): the particle-hole identity on every chain, and the fresh G of sampled
    chains (plus the chain with the largest identity residual) against the oracle.

    Bound of the G comparison (max |dG| / max(1, max |G|)): 1e-10, or 4x the spread between
    correct FP64 evaluations of the same G where that spread is larger -- the oracle with LAPACK's
    pivoted QR, the same with chunks of 5 slices, and the same with the pivots chosen from norms
    recomputed exactly (the GPU's rule; LAPACK downdates them).  At 20x20, U = 8, beta = 10 some
    fields have max |G| ~ 4e3, near-tied pivot norms, and such evaluations differ by ~1e-9.
    Identity on the GPU: 1e-8 relative (the oracle's own residual reaches ~1e-9 there)."""
    from oracle import Model, OracleChains
    w = di.WORKLOADS[name]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, qr_blocked=qr_blocked)
    seeds, fields = w.seeds(n_chains), w.fields(n_chains)
    b = dq.Batch(m, seeds, fields)
    g = b.debug_green(slice_, 0).cpu().numpy()
    D = di.staggered_sign(w.lattice, w.L)
    res = [_ph_residual(g[c], D) for c in range(n_chains)]
    assert max(res) < 1e-8, (name, int(np.argmax(res)), max(res))
    om = Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    alts = [Model(w.hopping(), w.U, w.dtau, w.n_slices, 5),
            Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, exact_pivot=True)]
    for c in sorted(set(sample) | {int(np.argmax(res))}):
        ref = OracleChains(om, fields[c:c + 1], seeds[c:c + 1]).debug_green(slice_, 0)[0]
        scale = max(1.0, float(np.max(np.abs(ref))))
        spread = 0.0
        for am in alts:
            alt = OracleChains(am, fields[c:c + 1], seeds[c:c + 1]).debug_green(slice_, 0)[0]
            spread = max(spread, float(np.max(np.abs(alt - ref))) / scale)
        err = float(np.max(np.abs(g[c] - ref))) / scale
        tol = max(1e-10, 4.0 * spread)
        print(f"{name} chain {c}: max|dG|/max(1,|G|) {err:.2e}, bar {tol:.2e} "
              f"(spread of correct FP64 evaluations {spread:.2e})")
        assert err < tol, (name, c, err, tol)
