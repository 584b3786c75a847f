"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: G and ratios on fixed fields to 1e-10 relative (max|dG| / max(1, max|G|), |dR|/|R|),
the Green's function of the FP64 path compared fresh and after at most stab_every wraps;
trajectories bitwise (fields) unless a decision was a near tie |u - R| < 1e-9, which the library
and the oracle both count; observables from the same final fields to 1e-9.
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


def oracle_for(w, n, first=0, fields=None):
    from oracle import Model, OracleChains
    m = Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    f = w.fields(n, first) if fields is None else fields
    return m, OracleChains(m, f, w.seeds(n, first))


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


# ------------------------------------------------------------------ building blocks
def test_mfma_lane_layout(dq):
    rng = np.random.default_rng(1)
    a = rng.standard_normal((16, 4))
    b = rng.standard_normal((4, 16))
    o64, o32 = dq.debug_mfma(a, b, a.astype(np.float32), b.astype(np.float32))
    assert np.allclose(o64.cpu().numpy(), a @ b, rtol=0, atol=1e-13)
    assert np.allclose(o32.cpu().numpy(), a.astype(np.float32) @ b.astype(np.float32), atol=1e-5)


def test_device_philox_matches_numpy(dq):
    for key, ctr in (((123, 456), (5, 6, 7, 8)), (((2 << 32) | 3, 0), (0, 0, 0, 0)),
                     ((2**64 - 1, 7), (2**64 - 9, 3, 0, 1))):
        out = dq.debug_philox(key, ctr, 16).cpu().numpy().astype(np.uint64)
        c = sum(int(w) << (64 * k) for k, w in enumerate(ctr))
        c = (c - 1) % (1 << 256)
        start = np.array([(c >> (64 * k)) & ((1 << 64) - 1) for k in range(4)], dtype=np.uint64)
        ref = np.random.Philox(counter=start, key=np.array(key, dtype=np.uint64)).random_raw(64)
        # numpy carries into word 1 on overflow of word 0; the device adds j to word 0 only,
        # so compare the blocks before any carry
        nb = 16 if ctr[0] + 16 < 2**64 else (2**64 - ctr[0])
        assert np.array_equal(out.reshape(-1)[:4 * nb], ref[:4 * nb])


@pytest.mark.parametrize("name", ["square4x4_U4_b2", "square8x8_U4_b4", "honeycomb6x6_U3_b6"])
def test_propagators(dq, name):
    from oracle import kinetic_propagators
    w = di.WORKLOADS[name]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    b = dq.Batch(m, w.seeds(1), w.fields(1))
    P = b.propagators().cpu().numpy()
    K, Ki = kinetic_propagators(w.hopping(), w.dtau)
    assert rel(P[0], K) < 1e-14 and rel(P[1], Ki) < 1e-14


def test_fields_from_seeds(dq):
    w = di.WORKLOADS["square8x8_U4_b4"]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    b = dq.Batch(m, w.seeds(6), None)
    assert np.array_equal(b.fields().cpu().numpy(), w.fields(6))


# ------------------------------------------------------------------ fixed-field parity
def wrap_spread(w, fields, l0, nw):
    """Spread of two correct FP64 evaluations of nw wraps from the fresh G(l0).

    One uses e^{-dtau T} from the eigendecomposition (the oracle), the other scipy's expm; the
    two propagators differ by ~1e-15 and the wraps amplify that roughly exponentially in nw.
    Returns max over chains and spins of max|dG| / max(1, max|G|).
    """
    import scipy.linalg as sla
    from oracle import Model
    m = Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    Kb, Kib = sla.expm(-w.dtau * w.hopping()), sla.expm(w.dtau * w.hopping())
    worst = 0.0
    for f in fields:
        for sg in (1, -1):
            G, _ = m.green(f, l0, sg)
            Ga, Gb = G.copy(), G.copy()
            for k in range(1, nw + 1):
                v = np.exp(sg * m.nu * f[l0 + k - 1].astype(float))
                Ga = m.wrap(Ga, f[l0 + k - 1], sg)
                Gb = v[:, None] * ((Kb @ Gb) @ Kib) / v[None, :]
            worst = max(worst, float(np.abs(Ga - Gb).max() / max(1.0, np.abs(Ga).max())))
    return worst


@pytest.mark.parametrize("name,n,cases", [
    ("square4x4_U4_b2", 2, [(0, 0), (0, 5), (10, 5), (20, 0), (7, 3), (0, 10), (10, 10)]),
    ("square8x8_U4_b4", 3, [(0, 0), (10, 0), (10, 5), (17, 3), (40, 0), (10, 10)]),
])
def test_debug_green_parity(dq, name, n, cases):
    """Fresh G and up to 5 wraps to 1e-10; 10 wraps within 10x the spread of two correct FP64
    evaluations (which itself reaches ~1e-10 there)."""
    w = di.WORKLOADS[name]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    f = w.fields(n)
    b = dq.Batch(m, w.seeds(n), f)
    _, oc = oracle_for(w, n)
    for sl, nw in cases:
        g = b.debug_green(sl, nw).cpu().numpy()
        ref = oc.debug_green(sl, nw)
        tol = 1e-10 if nw <= 5 else max(1e-10, 10.0 * wrap_spread(w, f, sl, nw))
        assert rel(g, ref) < tol, (sl, nw, rel(g, ref), tol)


@pytest.mark.parametrize("name,n", [("square4x4_U4_b2", 2), ("square8x8_U4_b4", 3)])
def test_debug_ratio_parity(dq, name, n):
    w = di.WORKLOADS[name]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    b = dq.Batch(m, w.seeds(n), w.fields(n))
    _, oc = oracle_for(w, n)
    for sl in (1, 10, 23 % w.n_slices + 1, w.n_slices):
        r = b.debug_ratios(sl).cpu().numpy()
        ref = oc.debug_ratios(sl)
        assert float(np.max(np.abs(r - ref) / np.abs(ref))) < 1e-10, sl


def test_initial_green_and_logdet(dq):
    w = di.WORKLOADS["square8x8_U4_b4"]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    b = dq.Batch(m, w.seeds(4), w.fields(4))
    obs, g = b.measure(green=True)
    _, oc = oracle_for(w, 4)
    assert rel(g.cpu().numpy(), oc.green()) < 1e-10
    ref = oc.measure()
    for c in range(4):
        assert math.isclose(obs["logdet_up"][c], ref[c]["logdet_up"], rel_tol=1e-11)
        assert math.isclose(obs["logdet_dn"][c], ref[c]["logdet_dn"], rel_tol=1e-11)
        assert abs(obs["double_occ"][c] - ref[c]["double_occ"]) < 1e-12


def test_spin_structure_form_factors(dq):
    """Structure factor at G(0) for the sublattice sign, a uniform and a real cos/sin form factor
    pair (S(Q) at a general Q is the sum of the two) against the oracle, to 1e-11."""
    from oracle import spin_structure
    w = di.WORKLOADS["square8x8_U4_b4"]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    b = dq.Batch(m, w.seeds(3), w.fields(3))
    _, oc = oracle_for(w, 3)
    g = oc.green()
    x = np.arange(64) % 8
    y = np.arange(64) // 8
    q = (2 * np.pi / 8) * np.array([1.0, 3.0])
    forms = [di.staggered_sign("square", 8), np.ones(64), np.cos(q[0] * x + q[1] * y),
             np.sin(q[0] * x + q[1] * y)]
    for f in forms:
        s = b.spin_structure(f).cpu().numpy()
        for c in range(3):
            ref = spin_structure(g[c, 0], g[c, 1], f)
            assert abs(s[c] - ref) < 1e-11 * max(1.0, abs(ref)), (c, s[c], ref)
    with pytest.raises(ValueError):
        b.spin_structure(np.ones(63))


# ------------------------------------------------------------------ trajectories
def _trajectory_check(dq, w, n, sweeps, delay_rank=0, first=0, qr_blocked=False):
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, delay_rank=delay_rank,
                      qr_blocked=qr_blocked)
    b = dq.Batch(m, w.seeds(n, first), w.fields(n, first))
    _, oc = oracle_for(w, n, first)
    b.sweep(sweeps)
    oc.sweep(sweeps)
    obs = b.measure()
    eps = di.staggered_sign(w.lattice, w.L)
    s_af = b.spin_structure(eps).cpu().numpy()
    ref = oc.measure(stagger=eps)
    f_gpu = b.fields().cpu().numpy()
    f_ref = oc.fields()
    for c in range(n):
        if obs["near_ties"][c] or ref[c]["near_ties"]:
            continue   # a legitimately ambiguous decision: the two may part ways
        assert np.array_equal(f_gpu[c], f_ref[c]), f"chain {c} trajectory differs"
        assert obs["accepted"][c] == ref[c]["accepted"]
        assert abs(obs["double_occ"][c] - ref[c]["double_occ"]) < 1e-9
        assert abs(obs["kinetic"][c] - ref[c]["kinetic"]) < 1e-9
        assert abs(s_af[c] - ref[c]["spin_af"]) < 1e-9
        assert math.isclose(obs["logdet_up"][c], ref[c]["logdet_up"], rel_tol=1e-9)
        assert obs["flags"][c] == 0
        assert obs["max_drift"][c] < 1e-6
    return b, obs


def test_trajectory_parity_square4x4(dq):
    w = di.WORKLOADS["square4x4_U4_b2"]
    b, obs = _trajectory_check(dq, w, 1, 100)
    assert obs["attempted"][0] == 100 * 20 * 16 and obs["sweeps_done"][0] == 100


def test_trajectory_parity_square8x8(dq):
    _trajectory_check(dq, di.WORKLOADS["square8x8_U4_b4"], 4, 3)


@pytest.mark.parametrize("k", [4, 8, 16])
def test_delay_rank_does_not_change_decisions(dq, k):
    _trajectory_check(dq, di.WORKLOADS["square8x8_U4_b4"], 2, 2, delay_rank=k, first=10)


def test_resume_is_bitwise(dq):
    w = di.WORKLOADS["square8x8_U4_b4"]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    a = dq.Batch(m, w.seeds(3), w.fields(3))
    a.sweep(4)
    b = dq.Batch(m, w.seeds(3), w.fields(3))
    b.sweep(2)
    b.sweep(2)
    oa, ga = a.measure(green=True)
    ob, gb = b.measure(green=True)
    assert np.array_equal(a.fields().cpu().numpy(), b.fields().cpu().numpy())
    assert np.array_equal(ga.cpu().numpy(), gb.cpu().numpy())


# ------------------------------------------------------------------ error paths
def test_rejects_bad_fields(dq):
    w = di.WORKLOADS["square4x4_U4_b2"]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    f = w.fields(2)
    f[1, 3, 5] = 0
    with pytest.raises(dq.DqmcError) as e:
        dq.Batch(m, w.seeds(2), f)
    assert e.value.status == -1


def test_rejects_small_workspace(dq):
    import torch
    w = di.WORKLOADS["square4x4_U4_b2"]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(dq.DqmcError) as e:
        dq.Batch(m, w.seeds(2), w.fields(2), workspace=ws)
    assert e.value.status == -2


# ------------------------------------------------------------------ other sizes
SQUARE6 = di.Workload("square6x6_U4_b2", 7, "square", 6, 4.0, 2.0, 0.1, 2, 2, 10)
SQUARE2 = di.Workload("square2x2_U4_b2", 8, "square", 2, 4.0, 2.0, 0.1, 2, 5, 5)
SQUARE12 = di.Workload("square12x12_U4_b2", 9, "square", 12, 4.0, 2.0, 0.1, 1, 1, 10)


@pytest.mark.parametrize("qr_blocked", [False, True])
def test_trajectory_parity_square12x12_two_level_delay(dq, qr_blocked):
    """N = 144: delay rank 32 with the accumulated panels (rank up to 128) flushed into G only
    when full and at the end of each slice (4.5 blocks per slice, a partial last block)."""
    b, _ = _trajectory_check(dq, SQUARE12, 1, 2, qr_blocked=qr_blocked)
    assert b.delay_rank == 32


def test_trajectory_parity_square2x2(dq):
    """N = 4, fewer sites than one delayed-update block."""
    _trajectory_check(dq, SQUARE2, 2, 5)


def test_trajectory_parity_square6x6_padded(dq):
    """N = 36 runs in the N <= 64 kernels padded to 64 (partial blocks, identity-padded inverse)."""
    b, _ = _trajectory_check(dq, SQUARE6, 2, 3)
    assert b.variant == 2


@pytest.mark.parametrize("qr_blocked", [False, True])
def test_trajectory_parity_honeycomb6x6_generic(dq, qr_blocked):
    """N = 72 (padded to 80) runs in the generic kernels, with the column-pivoted or the blocked
    stabilisation QR."""
    b, _ = _trajectory_check(dq, di.WORKLOADS["honeycomb6x6_U3_b6"], 1, 1, qr_blocked=qr_blocked)
    assert b.variant in (0, 1)


@pytest.mark.parametrize("name,cases,qr_blocked", [
    ("honeycomb12x12_U3_b6", [(0, 0), (30, 1), (60, 0)], False),
    ("honeycomb12x12_U3_b6", [(0, 0), (30, 1), (60, 0)], True),
    ("square20x20_U8_b10", [(0, 0), (50, 1), (100, 0)], False),
])
def test_large_lattice_green_parity(dq, name, cases, qr_blocked):
    """Fresh G and one wrap at N = 288 and N = 400 to 1e-10 relative (longer wrap sequences at
    these sizes differ between correct evaluations by more than that); the blocked QR where it
    applies (mildly graded products)."""
    w = di.WORKLOADS[name]
    m = dq.make_model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, qr_blocked=qr_blocked)
    b = dq.Batch(m, w.seeds(1), w.fields(1))
    _, oc = oracle_for(w, 1)
    for sl, nw in cases:
        g = b.debug_green(sl, nw).cpu().numpy()
        ref = oc.debug_green(sl, nw)
        assert rel(g, ref) < 1e-10, (name, sl, nw, rel(g, ref))


def test_qr_method_selection(dq):
    """The autotuner keeps the column-pivoted QR where the blocked one departs from it (20x20,
    U = 8, beta = 10: strongly graded products) and takes the blocked one at honeycomb 12x12,
    U = 3, beta = 6."""
    from paper_2106_00712_amd.autotune import Autotuner
    at = Autotuner()
    rec = {}
    for name in ("honeycomb12x12_U3_b6", "square20x20_U8_b10"):
        w = di.WORKLOADS[name]
        rec[name] = at.qr_method(w.hopping(), w.U, w.dtau, w.n_slices, w.fields(1), w.seeds(1),
                                 w.stab_every)
    assert rec["honeycomb12x12_U3_b6"]["qr_blocked"], rec
    assert not rec["square20x20_U8_b10"]["qr_blocked"], rec
