"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: an exact identity of the paper (SM section I.2),
a closed form, brute-force enumeration, the many-body Fock-space trace, particle-hole symmetry,
numpy's Philox, or high-precision arithmetic.
"""
import math

import numpy as np
import pytest

import dqmc_inputs as di
from oracle import (Model, OracleChains, hs_nu, philox4x64_10, accept_uniform, udt, udt_product,
                    measure_from_green)
import exact_tools as ex


# ------------------------------------------------------------------------- random numbers
@pytest.mark.parametrize("key,ctr", [((123, 456), (5, 6, 7, 8)), ((0, 0), (0, 0, 0, 0)),
                                     ((2**64 - 1, 7), (2**64 - 1, 3, 0, 1)),
                                     (((2 << 32) | 17, 0), (63, 39, 49, 1))])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox increments the 256-bit counter before each block.
    c = sum(int(w) << (64 * k) for k, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    start = [(c >> (64 * k)) & ((1 << 64) - 1) for k in range(4)]
    bg = np.random.Philox(counter=np.array(start, dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    assert tuple(int(v) for v in bg.random_raw(4)) == philox4x64_10(ctr, key)


def test_uniform_mapping():
    u = accept_uniform(99, 3, 2, 1)
    w = philox4x64_10((1, 2, 3, 1), (99, 0))[0]
    assert u == (w >> 11) / 2.0**53 and 0.0 <= u < 1.0


def test_seeded_fields_follow_philox_stream():
    seed, Lt, N = (2 << 32) | 5, 3, 7
    f = di.seeded_field(seed, Lt, N)
    for e in range(Lt * N):
        w = philox4x64_10((e // 4, 0, 0, 0), (seed, 0))[e % 4]
        assert f.reshape(-1)[e] == (1 if (w & 1) else -1)
    allf = di.WORKLOADS["square8x8_U4_b4"].fields(4)
    assert allf.shape == (4, 40, 64) and set(np.unique(allf)) == {-1, 1}
    assert abs(allf.mean()) < 0.05


# ------------------------------------------------------------------------- lattices
@pytest.mark.parametrize("L", [2, 4, 8])
def test_square_spectrum(L):
    k = 2 * np.pi * np.arange(L) / L
    eps = np.sort((-2.0 * (np.cos(k)[:, None] + np.cos(k)[None, :])).ravel())
    assert np.allclose(np.linalg.eigvalsh(di.square_hopping(L)), eps, atol=1e-12)


@pytest.mark.parametrize("L", [3, 6])
def test_honeycomb_spectrum(L):
    k = 2 * np.pi * np.arange(L) / L
    f = 1 + np.exp(1j * k)[:, None] + np.exp(1j * k)[None, :]
    eps = np.sort(np.concatenate([np.abs(f).ravel(), -np.abs(f).ravel()]))
    assert np.allclose(np.linalg.eigvalsh(di.honeycomb_hopping(L)), eps, atol=1e-12)


# ------------------------------------------------------------------------- HS and the weight
def test_hs_identity_on_all_occupations():
    """exp(-U dtau (n_up - 1/2)(n_dn - 1/2)) = 1/2 e^{-U dtau/4} sum_s e^{nu s (n_up - n_dn)}."""
    for U, dtau in ((4.0, 0.1), (8.0, 0.1), (3.0, 0.05), (3.83, 0.1)):
        nu = hs_nu(U, dtau)
        assert math.isclose(math.cosh(nu), math.exp(U * dtau / 2), rel_tol=1e-15)
        for nu_, nd in ex.all_occupation_states():
            lhs = math.exp(-U * dtau * (nu_ - 0.5) * (nd - 0.5))
            rhs = 0.5 * math.exp(-U * dtau / 4) * sum(math.exp(nu * s * (nu_ - nd)) for s in (1, -1))
            assert math.isclose(lhs, rhs, rel_tol=1e-14)


def test_nu_values():
    # cosh(nu) = e^{U dtau/2} inverted in closed form: nu = log(x + sqrt(x^2 - 1))
    for U in (3.0, 3.83, 4.0, 8.0):
        x = math.exp(U * 0.1 / 2)
        assert math.isclose(hs_nu(U, 0.1), math.log(x + math.sqrt(x * x - 1)), rel_tol=1e-14)


@pytest.mark.parametrize("n_slices,U", [(2, 4.0), (3, 8.0)])
def test_fock_trace_equals_hs_sum(n_slices, U):
    """Tr[(e^{-dtau H_U} e^{-dtau H_k})^L] = (e^{-U dtau/4}/2)^{N L} sum_s prod_sigma det(I + B)."""
    T = di.square_hopping(2)
    Zf, Df, Ef = ex.fock_trotter(T, U, 0.1, n_slices)
    Zh, Dh, Eh = ex.enumerate_observables(T, U, 0.1, n_slices)
    assert math.isclose(Zf, Zh, rel_tol=1e-12)
    assert math.isclose(Df, Dh, rel_tol=1e-11)
    assert math.isclose(Ef, Eh, rel_tol=1e-11)


def test_oracle_weight_and_green_vs_enumeration():
    """The oracle's stabilised G(0) and log det on every field of a 2x2, L=3 lattice."""
    T = di.square_hopping(2)
    m = Model(T, 4.0, 0.1, 3, 2)
    fields, w, Gu, Gd = ex.enumerate_fields(T, 4.0, 0.1, 3)
    for idx in range(0, fields.shape[0], 97):
        f = fields[idx].astype(np.int8)
        gu, ldu = m.green(f, 0, +1)
        gd, ldd = m.green(f, 0, -1)
        assert np.allclose(gu, Gu[idx], atol=1e-13) and np.allclose(gd, Gd[idx], atol=1e-13)
        assert math.isclose(ldu + ldd, math.log(w[idx]), rel_tol=1e-12, abs_tol=1e-12)


# ------------------------------------------------------------------------- closed forms
@pytest.mark.parametrize("lattice,L,beta,stab", [("square", 4, 2.0, 10), ("square", 8, 4.0, 10),
                                                 ("honeycomb", 6, 6.0, 10),
                                                 ("square", 2, 0.4, 2)])
def test_free_fermion_green(lattice, L, beta, stab):
    T = di.hopping(lattice, L)
    Lt = int(round(beta / 0.1))
    m = Model(T, 0.0, 0.1, Lt, stab)
    f = di.seeded_field(11, Lt, T.shape[0])
    G0 = ex.free_green(T, beta)
    for l in (0, stab, Lt // 2):
        G, _ = m.green(f, l, +1)
        # at U = 0 every slice propagator is exp(-dtau T): G(l) = G(0) for all l
        assert np.max(np.abs(G - G0)) < 1e-12
    assert np.allclose(np.diag(G0), 0.5, atol=1e-12)
    d, n, ek = measure_from_green(T, G0, G0)
    assert abs(d - 0.25) < 1e-12 and abs(n - 1.0) < 1e-12
    assert abs(ek - ex.free_kinetic(T, beta)) < 1e-12


def test_free_fermion_kinetic_energies():
    # U = 0 kinetic energies per site, recomputed from the spectrum of T
    for lattice, L, beta, val in (("square", 4, 2.0, -1.463692229945),
                                  ("square", 8, 4.0, -1.566637278560),
                                  ("honeycomb", 6, 6.0, -1.560884583917)):
        assert abs(ex.free_kinetic(di.hopping(lattice, L), beta) - val) < 1e-11


@pytest.mark.parametrize("U,L,beta", [(4.0, 4, 2.0), (4.0, 8, 4.0), (8.0, 4, 4.0)])
def test_uniform_field_green(U, L, beta):
    T = di.square_hopping(L)
    Lt = int(round(beta / 0.1))
    m = Model(T, U, 0.1, Lt, 10)
    f = np.ones((Lt, T.shape[0]), dtype=np.int8)
    for sigma in (+1, -1):
        G, _ = m.green(f, 0, sigma)
        Gx = ex.uniform_field_green(T, m.nu, Lt, beta, sigma)
        assert np.max(np.abs(G - Gx)) < 1e-12


# ------------------------------------------------------------------------- particle-hole
@pytest.mark.parametrize("lattice,L,beta,U", [("square", 4, 2.0, 4.0), ("square", 8, 4.0, 4.0),
                                              ("honeycomb", 3, 3.0, 3.0)])
def test_particle_hole_symmetry(lattice, L, beta, U):
    """mu = 0 on a bipartite lattice: G_dn = D (I - G_up^T) D, det(I+B_dn) = det(I+B_up) e^{-nu sum s}."""
    T = di.hopping(lattice, L)
    D = np.diag(di.staggered_sign(lattice, L))
    Lt = int(round(beta / 0.1))
    m = Model(T, U, 0.1, Lt, 10)
    f = di.seeded_field(5, Lt, T.shape[0])
    for l in (0, 10, Lt - 3):
        Gu, ldu = m.green(f, l, +1)
        Gd, ldd = m.green(f, l, -1)
        assert np.max(np.abs(Gd - D @ (np.eye(T.shape[0]) - Gu.T) @ D)) < 1e-10
        assert abs(ldd - (ldu - m.nu * float(f.sum()))) < 1e-9 * max(1.0, abs(ldu))
        # n_up + n_dn = 1 on every site, for every field
        assert np.allclose(np.diag(Gu) + np.diag(Gd), 1.0, atol=1e-10)
        if l > 0:
            ru, rd = m.ratios(Gu, Gd, f[l - 1])
            assert np.allclose(rd, ru * np.exp(2 * m.nu * f[l - 1]), rtol=1e-10)


# ------------------------------------------------------------------------- ratio, update, wrap
def _direct_green(m, f, l, sigma):
    """Unstabilised [I + B(l,0) B(L,l)]^{-1} by plain products (small beta only)."""
    N = m.N
    A = np.eye(N)
    for k in range(1, l + 1):
        A = m.B(f[k - 1], sigma) @ A
    Bb = np.eye(N)
    for k in range(l + 1, m.n_slices + 1):
        Bb = m.B(f[k - 1], sigma) @ Bb
    M = np.eye(N) + A @ Bb
    return np.linalg.inv(M), np.linalg.det(M)


def test_ratio_equals_determinant_ratio():
    T = di.square_hopping(4)
    m = Model(T, 4.0, 0.1, 10, 5)
    f = di.seeded_field(3, 10, 16)
    for l in (1, 4, 10):
        Gu, _ = m.green(f, l, +1)
        Gd, _ = m.green(f, l, -1)
        ru, rd = m.ratios(Gu, Gd, f[l - 1])
        _, du = _direct_green(m, f, l, +1)
        _, dd = _direct_green(m, f, l, -1)
        for i in range(16):
            g = f.copy()
            g[l - 1, i] = -g[l - 1, i]
            _, du2 = _direct_green(m, g, l, +1)
            _, dd2 = _direct_green(m, g, l, -1)
            assert math.isclose(ru[i], du2 / du, rel_tol=1e-10)
            assert math.isclose(rd[i], dd2 / dd, rel_tol=1e-10)


def test_sherman_morrison_matches_fresh_inverse():
    """The oracle's update path (wrap + Sherman-Morrison on every accept) against fresh inverses.

    Its drift record compares the wrapped and updated G with G rebuilt from the new fields at
    every stabilisation point; a wrong sign, index or factor in the update would show there.
    The rank-1 formula itself is checked against G (I + Delta (I - G))^{-1} by a linear solve.
    """
    T = di.square_hopping(4)
    m = Model(T, 4.0, 0.1, 20, 4)
    f = di.seeded_field(8, 20, 16)
    oc = OracleChains(m, f[None], [8])
    oc.sweep(2)
    st = oc.chains[0]
    assert st.max_drift < 1e-10 and st.accepted > 50 and st.max_logdet_err < 1e-10
    fu, _ = _direct_green(m, st.fields, 0, +1)
    assert np.max(np.abs(st.G[0] - fu)) < 1e-11
    # rank-1 update vs the definition through a solve, and vs the flipped field's fresh G
    l, i = 7, 5
    G, _ = _direct_green(m, st.fields, l, +1)
    s = float(st.fields[l - 1, i])
    d = math.exp(-2.0 * m.nu * s) - 1.0
    Dl = np.zeros((16, 16))
    Dl[i, i] = d
    G_def = G @ np.linalg.inv(np.eye(16) + Dl @ (np.eye(16) - G))
    g = st.fields.copy()
    g[l - 1, i] = -g[l - 1, i]
    G_new, _ = _direct_green(m, g, l, +1)
    assert np.max(np.abs(G_def - G_new)) < 1e-11


def test_wrap_matches_fresh():
    T = di.square_hopping(8)
    m = Model(T, 4.0, 0.1, 40, 10)
    f = di.seeded_field(13, 40, 64)
    G, _ = m.green(f, 10, +1)
    for w in range(1, 11):
        G = m.wrap(G, f[10 + w - 1], +1)
    G20, _ = m.green(f, 20, +1)
    assert np.max(np.abs(G - G20)) < 1e-10


def test_udt_factorisation():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((24, 24)) * np.logspace(0, 12, 24)[None, :]
    U, d, T = udt(X)
    assert np.allclose(U.T @ U, np.eye(24), atol=1e-14)
    assert np.allclose((U * d) @ T, X, rtol=0, atol=1e-14 * np.abs(X).max())
    assert np.all(d > 0) and np.all(np.diff(d) <= 1e-9 * d[:-1])   # pivoting sorts the scales


def test_green_vs_high_precision():
    """Stabilised G(0) of a strongly ill-conditioned product against 60-digit arithmetic."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    T = di.square_hopping(2)
    Lt, U = 100, 8.0
    m = Model(T, U, 0.1, Lt, 10)
    f = di.seeded_field(21, Lt, 4)
    lam, V = np.linalg.eigh(T)
    Vm = mpmath.matrix(V.tolist())
    K = Vm * mpmath.diag([mpmath.exp(-0.1 * mpmath.mpf(x)) for x in lam]) * Vm.T
    nu = mpmath.acosh(mpmath.exp(mpmath.mpf(U) * mpmath.mpf("0.1") / 2))
    for sigma in (+1, -1):
        P = mpmath.eye(4)
        for l in range(Lt):
            V_l = mpmath.diag([mpmath.exp(sigma * nu * int(s)) for s in f[l]])
            P = V_l * K * P
        Gx = (mpmath.eye(4) + P) ** -1
        G, ld = m.green(f, 0, sigma)
        err = max(abs(float(Gx[i, j]) - G[i, j]) for i in range(4) for j in range(4))
        # K enters both sides rounded to FP64; 100 slices of U=8 amplify that to ~1e-12
        assert err < 1e-11 * max(1.0, float(np.abs(G).max()))
        assert abs(float(mpmath.log(abs(mpmath.det(mpmath.eye(4) + P)))) - ld) < 1e-9


# ------------------------------------------------------------------------- chain behaviour
def test_resume_is_bitwise():
    T = di.square_hopping(4)
    m = Model(T, 4.0, 0.1, 20, 10)
    f = di.seeded_fields([1, 2], 20, 16)
    a = OracleChains(m, f, [1, 2])
    a.sweep(4)
    b = OracleChains(m, f, [1, 2])
    b.sweep(2)
    b.sweep(2)
    assert np.array_equal(a.fields(), b.fields())
    assert np.array_equal(a.green(), b.green())


def test_logdet_bookkeeping_and_drift():
    T = di.square_hopping(4)
    m = Model(T, 4.0, 0.1, 20, 10)
    oc = OracleChains(m, di.seeded_fields([7], 20, 16), [7])
    oc.sweep(3)
    o = oc.measure()[0]
    # ten wraps and ~100 rank-1 updates between refreshes from a random start: ~1e-9 drift
    assert o["max_logdet_err"] < 1e-8 and o["max_drift"] < 1e-8 and o["flags"] == 0
    assert o["attempted"] == 3 * 20 * 16 and 0 < o["accepted"] < o["attempted"]
    # log det from a plain determinant at this small beta
    _, du = _direct_green(m, oc.chains[0].fields, 0, +1)
    assert math.isclose(o["logdet_up"], math.log(du), rel_tol=1e-11)
    assert abs(o["density"] - 1.0) < 1e-10   # half filling holds field by field


@pytest.mark.slow
@pytest.mark.parametrize("sweep_mode", [0, 3])
def test_chain_statistics_match_enumeration(sweep_mode):
    """2x2, U=4, L_tau=4: oracle chains sample W(s); <D> and <E_k> within 4 sigma of exact, with
    up sweeps only and with alternating up/down sweeps (then also the per-slice estimators)."""
    T = di.square_hopping(2)
    Lt = 4
    _, Dx, Ex = ex.enumerate_observables(T, 4.0, 0.1, Lt)
    m = Model(T, 4.0, 0.1, Lt, 2, sweep_mode=sweep_mode)
    n_chains, burn, n_meas = 24, 20, 150
    seeds = list(range(100, 100 + n_chains))
    oc = OracleChains(m, di.seeded_fields(seeds, Lt, 4), seeds)
    oc.sweep(burn)
    start = [(o["slice_double_occ"] * o["slice_meas"], o["slice_kinetic"] * o["slice_meas"],
              o["slice_meas"]) for o in oc.measure()]
    sums = np.zeros((n_chains, 2))
    for _ in range(n_meas):
        oc.sweep(1)
        for c, o in enumerate(oc.measure()):
            sums[c] += (o["double_occ"], o["kinetic"])
    means = sums / n_meas
    checks = [(means[:, 0], Dx), (means[:, 1], Ex)]
    if sweep_mode & 2:
        end = oc.measure()
        per_slice = np.array([[(o["slice_double_occ"] * o["slice_meas"] - a) / (o["slice_meas"] - n),
                               (o["slice_kinetic"] * o["slice_meas"] - b) / (o["slice_meas"] - n)]
                              for o, (a, b, n) in zip(end, start)])
        assert all(o["slice_meas"] == (burn + n_meas) * Lt for o in end)
        checks += [(per_slice[:, 0], Dx), (per_slice[:, 1], Ex)]
    for v, exact in checks:
        mu, se = v.mean(), v.std(ddof=1) / math.sqrt(n_chains)
        assert abs(mu - exact) < 4 * se + 1e-12, (mu, se, exact)


def test_unwrap_equals_fresh_green():
    """Down sweeps move G(l) to G(l-1) = B_l^{-1} G(l) B_l: equal to the fresh G(l-1)."""
    w = di.WORKLOADS["square4x4_U4_b2"]
    m = Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    f = w.fields(1)[0]
    for l in (1, 7, 20):
        for sigma in (+1, -1):
            G, _ = m.green(f, l, sigma)
            ref, _ = m.green(f, l - 1, sigma)
            assert np.max(np.abs(m.unwrap(G, f[l - 1], sigma) - ref)) < 1e-11


def test_alternating_sweeps_stay_on_the_fresh_green():
    """Up then down sweeps on 4x4: every stabilisation replaces a running G within 1e-9 of the
    fresh one (a wrong unwrap or slice order would drift at once), the chain ends at G(0)."""
    w = di.WORKLOADS["square4x4_U4_b2"]
    m = Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, sweep_mode=3)
    oc = OracleChains(m, w.fields(2), w.seeds(2))
    oc.sweep(4)
    for c, o in enumerate(oc.measure()):
        assert o["max_drift"] < 1e-9 and o["flags"] == 0
        assert o["slice_meas"] == 4 * w.n_slices
        f = oc.fields()[c]
        assert np.max(np.abs(oc.green()[c, 0] - m.green(f, 0, +1)[0])) < 1e-12


def test_per_slice_estimators_free_fermions():
    """U = 0: every field gives the free G at every slice, so the per-slice averages equal the
    closed forms D = 1/4 and the free kinetic energy."""
    T = di.square_hopping(4)
    m = Model(T, 0.0, 0.1, 20, 10, sweep_mode=3)
    oc = OracleChains(m, di.seeded_fields([3], 20, 16), [3])
    oc.sweep(2)
    o = oc.measure()[0]
    assert abs(o["slice_double_occ"] - 0.25) < 1e-12
    assert abs(o["slice_kinetic"] - ex.free_kinetic(T, 2.0)) < 1e-12


# ------------------------------------------------------------------ spin structure factor
@pytest.mark.parametrize("form", ["staggered", "uniform", "random"])
def test_spin_structure_equals_fock_trace(form):
    """The Wick estimator averaged over all HS fields of a 2x2 lattice equals the Fock-space trace
    of (1/N)(sum f s^z)^2: staggered f = (-1)^(x+y), uniform f = 1, and a random real f (which
    tells the f^2 weight of the diagonal term from a plain trace)."""
    from oracle import spin_structure
    T = di.square_hopping(2)
    eps = {"staggered": di.staggered_sign("square", 2), "uniform": np.ones(4),
           "random": np.random.default_rng(5).uniform(-1.5, 1.5, 4)}[form]
    U, dtau, Lt = 4.0, 0.1, 3
    fields, w, Gu, Gd = ex.enumerate_fields(T, U, dtau, Lt)
    vals = np.array([spin_structure(Gu[k], Gd[k], eps) for k in range(fields.shape[0])])
    hs = float(np.sum(w * vals) / np.sum(w))
    fock = ex.fock_trotter(T, U, dtau, Lt, form=eps)[3]
    assert math.isclose(hs, fock, rel_tol=1e-11), (hs, fock)


def test_spin_structure_free_fermions():
    """U = 0: G^up = G^dn = G free, so m = 0 and S = (1/(4N)) 2 (tr G - sum eps eps G_ij G_ji);
    on the 4x4 lattice at beta = 2 the uniform S(Gamma) equals the free-fermion value of
    (1/N)<(S^z)^2> = (1/(2N)) sum_k f_k (1 - f_k) (one-body modes, both spins)."""
    from oracle import spin_structure
    T = di.square_hopping(4)
    G = ex.free_green(T, 2.0)
    lam = np.linalg.eigvalsh(T)
    f = 1.0 / (1.0 + np.exp(2.0 * lam))
    ref = float(np.sum(f * (1 - f))) / (2 * 16)
    assert math.isclose(spin_structure(G, G, np.ones(16)), ref, rel_tol=1e-12)


# ------------------------------------------------------------------ exact-norm pivoting
def test_udt_exact_pivot_is_a_pivoted_udt():
    """X = U D T with U orthogonal and, column-pivoted QR's defining property, every entry of
    T' = D^-1 S R at most 1 in size (|R_jj| >= |R_ij|); on a graded random matrix."""
    from oracle import udt_exact_pivot
    rng = np.random.default_rng(11)
    X = rng.standard_normal((40, 40)) @ np.diag(np.exp(rng.uniform(-25, 25, 40)))
    U, d, T = udt_exact_pivot(X)
    assert np.max(np.abs(U.T @ U - np.eye(40))) < 1e-13
    rec = (U * d[None, :]) @ T
    assert np.max(np.abs(rec - X) / np.abs(X).max(axis=0)[None, :]) < 1e-13
    assert np.max(np.abs(T)) <= 1.0 + 1e-12
    assert np.all(d[:-1] >= d[1:] * (1 - 1e-12))     # the pivoted diagonal does not increase


def test_udt_exact_pivot_matches_lapack_when_norms_separate():
    """With well separated column norms both pivot rules take the same columns: the same U, d, T
    as LAPACK's pivoted QR to rounding."""
    from oracle import udt, udt_exact_pivot
    rng = np.random.default_rng(12)
    # a well-conditioned matrix with its columns scaled a factor ~3 apart, in shuffled order
    B = np.eye(30) + 0.1 * rng.standard_normal((30, 30))
    X = (B * (10.0 ** (-np.arange(30) / 2.0))[None, :])[:, rng.permutation(30)]
    a, b = udt(X), udt_exact_pivot(X)
    for u, v in zip(a, b):
        assert np.max(np.abs(u - v)) < 1e-10 * max(1.0, np.max(np.abs(u)))


def test_exact_pivot_green_matches_lapack_green():
    """Fresh G by the exact-norm variant equals the LAPACK-pivoted oracle on a mildly graded
    workload (honeycomb 6x6, U = 3, beta = 6) to 1e-11."""
    from oracle import Model
    w = di.WORKLOADS["honeycomb6x6_U3_b6"]
    f = w.fields(1)[0]
    a = Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every)
    b = Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, exact_pivot=True)
    for l in (0, 30):
        ga, la = a.green(f, l, +1)
        gb, lb = b.green(f, l, +1)
        assert np.max(np.abs(ga - gb)) < 1e-11 and abs(la - lb) < 1e-9


# ------------------------------------------------------------------------- baseline mode
@pytest.mark.parametrize("lattice,L,beta,U,stab,sweep_mode,sweeps", [
    ("square", 4, 2.0, 4.0, 10, 0, 4),      # L_tau a multiple of n_s
    ("square", 4, 2.0, 4.0, 7, 0, 3),       # ragged top chunk (20 = 7 + 7 + 6)
    ("square", 4, 2.0, 4.0, 10, 1, 4),      # alternating sweeps reuse the other direction's stack
    ("square", 4, 2.0, 4.0, 7, 3, 3),
    ("honeycomb", 2, 1.5, 3.0, 4, 1, 3),
])
def test_baseline_mode_matches_reference(lattice, L, beta, U, stab, sweep_mode, sweeps):
    """Stacked factors (right stack per up sweep or from the down sweep before, running left
    factors) give the fresh G that rebuilding both products from scratch gives, so the chains
    take the same decisions; the reference mode is the one pinned by the tests above."""
    T = di.hopping(lattice, L)
    n_sl = int(round(beta / 0.1))
    seeds = [11, 12]
    f = di.seeded_fields(seeds, n_sl, T.shape[0])
    ref = OracleChains(Model(T, U, 0.1, n_sl, stab, sweep_mode=sweep_mode), f, seeds)
    base = OracleChains(Model(T, U, 0.1, n_sl, stab, sweep_mode=sweep_mode, stacks=True), f, seeds)
    ref.sweep(sweeps)
    base.sweep(sweeps)
    assert np.array_equal(ref.fields(), base.fields())
    assert np.max(np.abs(ref.green() - base.green())) < 1e-10
    for a, b in zip(ref.measure(), base.measure()):
        assert a["accepted"] == b["accepted"] and a["flags"] == b["flags"] == 0
        assert abs(a["logdet_up"] - b["logdet_up"]) < 1e-9 and abs(a["logdet_dn"] - b["logdet_dn"]) < 1e-9
        assert abs(a["max_drift"] - b["max_drift"]) < 1e-10


def test_baseline_mode_8x8():
    w = di.WORKLOADS["square8x8_U4_b4"]
    f, s = w.fields(2), w.seeds(2)
    ref = OracleChains(Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every), f, s)
    base = OracleChains(Model(w.hopping(), w.U, w.dtau, w.n_slices, w.stab_every, stacks=True), f, s)
    ref.sweep(2)
    base.sweep(2)
    assert np.array_equal(ref.fields(), base.fields())
    assert np.max(np.abs(ref.green() - base.green())) < 1e-10
