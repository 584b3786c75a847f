"""FP64 CPU oracle for DQMC sweeps of the Hubbard model: many short, independent chains.

TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference that the HIP path is checked
against.  Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may import
it; the product library never does, and this module imports nothing from the product package.

What is computed, in the paper's notation (supplement section I.2, "Determinant Quantum Monte
Carlo"; the NIMC scheme, Alg. 1 step 4, runs one such chain per starting configuration):
  * beta is cut into L_tau slices of width dtau (Trotter-Suzuki split of Z);
  * the Hubbard interaction is decoupled by a discrete HS field s_{i,l} = +-1 with
    cosh(nu) = exp(U dtau / 2);
  * the slice propagator is B^sigma_l = exp(sigma nu Diag{s_{.,l}}) exp(-dtau T), sigma = +1 (up),
    -1 (down), and B^sigma(l2, l1) = B_{l2} ... B_{l1+1};
  * a field configuration has weight W(s) proportional to prod_sigma det[I + B^sigma(L_tau, 0)].
The sweep itself (equal-time Green's function, wrap, single-flip Metropolis ratio,
Sherman-Morrison update, stabilised products) is the textbook DQMC that the paper cites for
this construction; every step below is derived from the weight above, in the function doing it.

Readings where the paper is silent (listed with reasons in the design notes):
  * B has the HS factor on the left of exp(-dtau T), as in the definition of B^sigma(l2, l1);
  * Metropolis acceptance: draw u in [0, 1), accept iff u < R, one uniform per attempt;
  * a sweep visits slices l = 1 .. L_tau in ascending order and sites i = 0 .. N-1 in each;
  * stabilisation (fresh G from column-pivoted QR products) after slice l whenever
    l % stab_every == 0 and after l = L_tau; the wrapped G is replaced by the fresh one;
  * measurements use the fresh G(L_tau) = G(0) left after the last sweep.

Two ways to obtain the fresh G at a stabilisation point, the same products in the same chunks:
  * reference mode (default): both B products rebuilt from slice 1 and from slice L_tau at every
    stabilisation point, the simplest form to trust;
  * baseline mode (Model.stacks = True): the UDT factors of B(L_tau, p_j)^T at the points
    p_j = min(j n_s, L_tau) kept as a stack built once per up sweep (or by the preceding down
    sweep when sweeps alternate), and B(p_j, 0) pushed one chunk at a time onto a running left
    factorisation: the algorithm class of the GPU path, used to time the oracle.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field
from typing import List, Optional, Tuple

import numpy as np
import scipy.linalg as sla

from .philox import accept_uniform

NEAR_TIE = 1e-9          # |u - R| below this marks a decision that rounding could flip
FLAG_NONFINITE = 1
FLAG_NEGATIVE_RATIO = 2
FLAG_DRIFT = 4
DRIFT_LIMIT = 1e-3


# ------------------------------------------------------------------------------------ model
def hs_nu(U: float, dtau: float) -> float:
    """HS coupling: cosh(nu) = exp(U dtau / 2) (discrete HS transformation, SM section I.2)."""
    return math.acosh(math.exp(0.5 * U * dtau))


def kinetic_propagators(T: np.ndarray, dtau: float, mu: float = 0.0):
    """exp(-dtau (T - mu)) and its inverse exp(+dtau (T - mu)) from the eigenvectors of T."""
    lam, V = np.linalg.eigh(T - mu * np.eye(T.shape[0]))
    return (V * np.exp(-dtau * lam)) @ V.T, (V * np.exp(dtau * lam)) @ V.T


def slice_B(expK: np.ndarray, nu: float, s_l: np.ndarray, sigma: int) -> np.ndarray:
    """B^sigma_l = exp(sigma nu Diag{s_l}) exp(-dtau T)."""
    return np.exp(sigma * nu * s_l.astype(np.float64))[:, None] * expK


def slice_Binv(expKinv: np.ndarray, nu: float, s_l: np.ndarray, sigma: int) -> np.ndarray:
    """(B^sigma_l)^{-1} = exp(+dtau T) exp(-sigma nu Diag{s_l})."""
    return expKinv * np.exp(-sigma * nu * s_l.astype(np.float64))[None, :]


# ------------------------------------------------------------------------ stabilised products
def udt(X: np.ndarray):
    """X = U Diag(d) T with U orthogonal, d > 0, from column-pivoted Householder QR (LAPACK).

    X P = Q R; d = |diag R|; the signs of diag R move into U; T = Diag(d)^{-1} S R P^T.
    """
    Q, R, piv = sla.qr(X, pivoting=True)
    r = np.diag(R)
    sgn = np.where(r < 0.0, -1.0, 1.0)
    d = np.abs(r)
    U = Q * sgn[None, :]
    Rn = (sgn[:, None] * R) / d[:, None]
    T = np.empty_like(Rn)
    T[:, piv] = Rn
    return U, d, T


def udt_exact_pivot(X: np.ndarray):
    """As udt, with the pivot of every step chosen from the column norms recomputed exactly on
    the partly reduced matrix (LAPACK's pivoted QR downdates them instead).  Both rules take the
    largest remaining norm; they part only where remaining norms tie to rounding, and then give
    different, equally valid factorisations.  Plain Householder steps:
      column j: x = A[j:, pivot], alpha = -sign(x_0) |x|, v = x - alpha e_0,
      beta = 1 / (alpha (alpha - x_0)), A[j:, j:] <- (I - beta v v^T) A[j:, j:];
    Q = H_0 ... H_{n-1} applied to I from the last reflector back."""
    A = np.array(X, dtype=np.float64, copy=True)
    n = A.shape[1]
    piv = np.arange(n)
    refl = []
    for j in range(n):
        nrm = np.sum(A[j:, j:] ** 2, axis=0)
        p = j + int(np.argmax(nrm))
        A[:, [j, p]] = A[:, [p, j]]
        piv[[j, p]] = piv[[p, j]]
        x = A[j:, j].copy()
        nx = float(np.sqrt(np.sum(x * x)))
        alpha = -nx if x[0] >= 0.0 else nx
        v = x.copy()
        v[0] -= alpha
        beta = 1.0 / (alpha * (alpha - x[0])) if nx > 0.0 else 0.0
        A[j:, j:] -= beta * np.outer(v, v @ A[j:, j:])
        refl.append((v, beta))
    R = np.triu(A)
    Q = np.eye(A.shape[0])
    for j in range(n - 1, -1, -1):
        v, beta = refl[j]
        Q[j:, :] -= beta * np.outer(v, v @ Q[j:, :])
    r = np.diag(R)
    sgn = np.where(r < 0.0, -1.0, 1.0)
    d = np.abs(r)
    U = Q * sgn[None, :]
    Rn = (sgn[:, None] * R) / d[:, None]
    T = np.empty_like(Rn)
    T[:, piv] = Rn
    return U, d, T


def udt_product(factors: List[np.ndarray], chunk: int, n: int, factorise=None):
    """UDT of factors[-1] @ ... @ factors[0] (n x n), re-factorised after every `chunk` factors.

    Each chunk is multiplied onto U Diag(d) and factorised again; the new T' multiplies the
    accumulated T from the left.  The scales of the product live only in d.  No factors: I.
    `factorise` is udt (LAPACK's pivoted QR) unless another UDT routine is given.
    """
    factorise = factorise or udt
    U, d, T = np.eye(n), np.ones(n), np.eye(n)
    for start in range(0, len(factors), chunk):
        X = U * d[None, :]
        for F in factors[start:start + chunk]:
            X = F @ X
        U, d, Tn = factorise(X)
        T = Tn @ T
    return U, d, T


def udt_push(fac, factors: List[np.ndarray], factorise=None):
    """UDT of (factors[-1] @ ... @ factors[0]) @ U Diag(d) T for fac = (U, d, T): the chunk is
    multiplied onto U Diag(d) and factorised again, the new T' multiplies T from the left (one
    chunk of udt_product)."""
    factorise = factorise or udt
    U, d, T = fac
    X = U * d[None, :]
    for F in factors:
        X = F @ X
    Un, dn, Tn = factorise(X)
    return Un, dn, Tn @ T


def green_two_sided(left, right_t):
    """G = [I + A B]^{-1} with A = UL DL TL and B^T = UR DR TR, and log|det(I + A B)|.

    Split every scale vector at 1: d = d_big * d_small with d_big = max(d, 1), d_small =
    min(d, 1).  Then, U being orthogonal,
        I + A B = UL DLb [DLb^{-1} UL^T UR DRb^{-1} + DLs TL TR^T DRs] DRb UR^T,
    so with M the bracket, G = UR DRb^{-1} M^{-1} DLb^{-1} UL^T and
    log|det(I + A B)| = sum log DLb + sum log DRb + log|det M|.
    """
    UL, dL, TL = left
    UR, dR, TR = right_t
    dLb, dLs = np.maximum(dL, 1.0), np.minimum(dL, 1.0)
    dRb, dRs = np.maximum(dR, 1.0), np.minimum(dR, 1.0)
    M = (UL.T @ UR) / dLb[:, None] / dRb[None, :] + dLs[:, None] * (TL @ TR.T) * dRs[None, :]
    rhs = UL.T / dLb[:, None]
    G = UR @ (np.linalg.solve(M, rhs) / dRb[:, None])
    _, logabs = np.linalg.slogdet(M)
    return G, float(np.sum(np.log(dLb)) + np.sum(np.log(dRb)) + logabs)


# -------------------------------------------------------------------------------- the model
@dataclass
class Model:
    T: np.ndarray
    U: float
    dtau: float
    n_slices: int
    stab_every: int
    mu: float = 0.0
    exact_pivot: bool = False   # UDT by udt_exact_pivot instead of LAPACK's pivoted QR
    sweep_mode: int = 0         # bit 0: alternate up and down sweeps; bit 1: per-slice measurements
    stacks: bool = False        # baseline mode: stacked UDT factors instead of rebuilt products

    def __post_init__(self):
        self.T = np.asarray(self.T, dtype=np.float64)
        self.N = self.T.shape[0]
        self.nu = hs_nu(self.U, self.dtau)
        self.expK, self.expKinv = kinetic_propagators(self.T, self.dtau, self.mu)

    def B(self, s_l, sigma):
        return slice_B(self.expK, self.nu, s_l, sigma)

    def Binv(self, s_l, sigma):
        return slice_Binv(self.expKinv, self.nu, s_l, sigma)

    def green(self, fields: np.ndarray, l: int, sigma: int):
        """Fresh equal-time G^sigma(l) = [I + B(l, 0) B(L_tau, l)]^{-1} and log|det(I + B(L_tau,0))|.

        Both products are rebuilt from scratch: B(l, 0) from slice 1 upwards and B(L_tau, l)^T
        = B_{l+1}^T ... B_{L_tau}^T from slice L_tau downwards, each in chunks of stab_every.
        """
        Lt = self.n_slices
        fac = udt_exact_pivot if self.exact_pivot else udt
        left = udt_product([self.B(fields[k - 1], sigma) for k in range(1, l + 1)],
                           self.stab_every, self.N, fac)
        right_t = udt_product([self.B(fields[k - 1], sigma).T for k in range(Lt, l, -1)],
                              self.stab_every, self.N, fac)
        return green_two_sided(left, right_t)

    def points(self):
        """Stabilisation points p_j = min(j n_s, L_tau), j = 0 .. J."""
        J = -(-self.n_slices // self.stab_every)
        return [min(j * self.stab_every, self.n_slices) for j in range(J + 1)]

    def _factorise(self):
        return udt_exact_pivot if self.exact_pivot else udt

    def left_chunk(self, fac, fields, lo: int, hi: int, sigma: int):
        """B(hi, lo) B(lo, 0) from the factors of B(lo, 0): push B_{lo+1}, ..., B_hi."""
        return udt_push(fac, [self.B(fields[k - 1], sigma) for k in range(lo + 1, hi + 1)],
                        self._factorise())

    def right_chunk(self, fac, fields, lo: int, hi: int, sigma: int):
        """B(L_tau, lo)^T = B(hi, lo)^T B(L_tau, hi)^T from the factors of B(L_tau, hi)^T:
        push B_hi^T, ..., B_{lo+1}^T."""
        return udt_push(fac, [self.B(fields[k - 1], sigma).T for k in range(hi, lo, -1)],
                        self._factorise())

    def identity_udt(self):
        return np.eye(self.N), np.ones(self.N), np.eye(self.N)

    def wrap(self, G, s_l, sigma):
        """G(l) = B_l G(l-1) B_l^{-1}: [I + B(l,0)B(L,l)]^{-1} conjugated by B_l."""
        return self.B(s_l, sigma) @ G @ self.Binv(s_l, sigma)

    def unwrap(self, G, s_l, sigma):
        """G(l-1) = B_l^{-1} G(l) B_l, the wrap run backwards (down sweeps)."""
        return self.Binv(s_l, sigma) @ G @ self.B(s_l, sigma)

    def ratios(self, G_up, G_dn, s_l):
        """Per-site ratios for flipping s_{i,l} alone, given G(l) of both spins.

        The flip multiplies B^sigma_l from the left by I + Delta^sigma with Delta^sigma =
        (exp(-2 sigma nu s_{i,l}) - 1) e_i e_i^T.  With G = [I + A]^{-1}, A = B(l,0)B(L,l):
        det(I + (I+Delta)A) / det(I + A) = det(I + Delta (I - G)) = 1 + Delta_ii (1 - G_ii).
        """
        s = s_l.astype(np.float64)
        d_up = np.exp(-2.0 * self.nu * s) - 1.0
        d_dn = np.exp(+2.0 * self.nu * s) - 1.0
        return 1.0 + d_up * (1.0 - np.diag(G_up)), 1.0 + d_dn * (1.0 - np.diag(G_dn))


def measure_from_green(T: np.ndarray, G_up: np.ndarray, G_dn: np.ndarray):
    """Equal-time estimators for one field (Wick's theorem; spins factorise at fixed field).

    <n_{i sigma}> = 1 - G_ii; double occupancy (1/N) sum_i <n_up n_dn> = (1/N) sum_i
    (1 - G^up_ii)(1 - G^dn_ii); density (1/N) sum_i (2 - G^up_ii - G^dn_ii); kinetic energy per
    site (1/N) sum_sigma sum_ij T_ij <c^+_i c_j> = (1/N) sum_sigma sum_ij T_ij (delta_ij - G_ji).
    """
    N = T.shape[0]
    gu, gd = np.diag(G_up), np.diag(G_dn)
    docc = float(np.sum((1.0 - gu) * (1.0 - gd)) / N)
    dens = float(np.sum(2.0 - gu - gd) / N)
    kin = 0.0
    for G in (G_up, G_dn):
        kin += float(np.sum(T * (np.eye(N) - G.T)))
    return docc, dens, kin / N


def spin_structure(G_up: np.ndarray, G_dn: np.ndarray, form: np.ndarray) -> float:
    """(1/N) sum_ij f_i f_j <s^z_i s^z_j> for one field, s^z_i = (n_i,up - n_i,dn)/2, with a real
    form factor f (the magnetic structure factor S(Q) of the paper's loss function, main text
    eq. (4): with phases f_i = +-1 it is S(Q) at a wave vector whose phases are real, e.g. the
    sublattice sign for honeycomb S(Gamma); a complex phase e^{iQ.r} splits into f = cos and
    f = sin, and S(Q) is the sum of the two).

    Wick's theorem at fixed field, spins independent:
      <n_i,s n_j,s'> = (1 - G^s_ii)(1 - G^s'_jj) + delta_ss' (delta_ij - G^s_ji) G^s_ij,
    so with m = sum_i f_i (G^dn_ii - G^up_ii)
      (1/N) sum_ij f_i f_j <s^z_i s^z_j>
        = (1/(4N)) [ m^2 + sum_s ( sum_i f_i^2 G^s_ii - sum_ij f_i f_j G^s_ij G^s_ji ) ].
    """
    N = G_up.shape[0]
    f = np.asarray(form, dtype=np.float64)
    m = float(np.sum(f * (np.diag(G_dn) - np.diag(G_up))))
    tot = m * m
    for G in (G_up, G_dn):
        tot += float(np.sum(f * f * np.diag(G))) - float(np.sum(np.outer(f, f) * G * G.T))
    return tot / (4.0 * N)


# -------------------------------------------------------------------------------- chains
@dataclass
class ChainState:
    fields: np.ndarray                 # int8 [L_tau][N], modified in place by sweeps
    seed: int
    sweeps_done: int = 0
    G: List[np.ndarray] = dc_field(default_factory=list)   # [G_up, G_dn] = G(0)
    logdet: List[float] = dc_field(default_factory=lambda: [0.0, 0.0])
    attempted: int = 0
    accepted: int = 0
    near_ties: int = 0
    max_drift: float = 0.0
    max_logdet_err: float = 0.0
    flags: int = 0
    slice_docc: float = 0.0            # sums of the per-slice equal-time estimators
    slice_kin: float = 0.0
    slice_meas: int = 0
    # baseline mode: per spin, factors of B(p_j, 0) (left) and B(L_tau, p_j)^T (right) by j
    left: List[dict] = dc_field(default_factory=lambda: [{}, {}])
    right: List[dict] = dc_field(default_factory=lambda: [{}, {}])
    right_valid: bool = False


class OracleChains:
    """A batch of independent chains on one model, with the semantics of init / sweep / measure."""

    def __init__(self, model: Model, fields: np.ndarray, seeds):
        self.m = model
        fields = np.asarray(fields)
        if fields.ndim == 2:
            fields = fields[None]
        if fields.shape[1:] != (model.n_slices, model.N):
            raise ValueError("fields must be [n_chains][n_slices][N]")
        if not np.all(np.abs(fields) == 1):
            raise ValueError("fields must be +-1")
        self.chains = []
        for c in range(fields.shape[0]):
            st = ChainState(fields=fields[c].astype(np.int8).copy(), seed=int(seeds[c]))
            for k, sigma in enumerate((+1, -1)):
                G, ld = model.green(st.fields, 0, sigma)
                st.G.append(G)
                st.logdet[k] = ld
            self.chains.append(st)

    # -- one sweep of one chain ---------------------------------------------------------
    def _metropolis_slice(self, st: ChainState, G_up, G_dn, l: int, logdet_run):
        """Attempt every site of slice l (sites ascending) with G = G(l) of both spins."""
        m = self.m
        s_l = st.fields[l - 1]
        for i in range(m.N):
            s = float(s_l[i])
            d_up = math.exp(-2.0 * m.nu * s) - 1.0
            d_dn = math.exp(+2.0 * m.nu * s) - 1.0
            r_up = 1.0 + d_up * (1.0 - G_up[i, i])
            r_dn = 1.0 + d_dn * (1.0 - G_dn[i, i])
            R = r_up * r_dn
            u = accept_uniform(st.seed, st.sweeps_done, l - 1, i)
            st.attempted += 1
            if not math.isfinite(R):
                st.flags |= FLAG_NONFINITE
                continue
            if R < 0.0:
                st.flags |= FLAG_NEGATIVE_RATIO
                continue
            if abs(u - R) < NEAR_TIE:
                st.near_ties += 1
            if u < R:
                # Sherman-Morrison: G' = G (I + Delta (I - G))^{-1}
                #                      = G - (Delta / R_sigma) G[:, i] (e_i - G[i, :])
                for k, (d, r) in enumerate(((d_up, r_up), (d_dn, r_dn))):
                    G = G_up if k == 0 else G_dn
                    col = G[:, i].copy()
                    row = -G[i, :].copy()
                    row[i] += 1.0
                    G -= (d / r) * np.outer(col, row)
                logdet_run[0] += math.log(abs(r_up))
                logdet_run[1] += math.log(abs(r_dn))
                s_l[i] = -s_l[i]
                st.accepted += 1
        if m.sweep_mode & 2:
            docc, _, kin = measure_from_green(m.T, G_up, G_dn)
            st.slice_docc += docc
            st.slice_kin += kin
            st.slice_meas += 1

    def _fresh(self, st: ChainState, l: int, k: int, sigma: int):
        """Fresh G^sigma(l) and log|det|: rebuilt from scratch (reference mode) or from the left
        and right factors at stabilisation point l (baseline mode)."""
        if not self.m.stacks:
            return self.m.green(st.fields, l, sigma)
        j = self.m.points().index(l)
        return green_two_sided(st.left[k][j], st.right[k][j])

    def _stabilise(self, st: ChainState, Gs, l: int, logdet_run):
        """Replace the running G(l) of both spins by the fresh one; record drift and log-det error."""
        for k, sigma in enumerate((+1, -1)):
            G_new, ld = self._fresh(st, l, k, sigma)
            drift = float(np.max(np.abs(Gs[k] - G_new)))
            if not math.isfinite(drift):
                st.flags |= FLAG_NONFINITE
            st.max_drift = max(st.max_drift, drift)
            st.max_logdet_err = max(st.max_logdet_err, abs(ld - logdet_run[k]))
            logdet_run[k] = ld
            Gs[k] = G_new
        if st.max_drift > DRIFT_LIMIT:
            st.flags |= FLAG_DRIFT

    def _build_right(self, st: ChainState):
        """Baseline mode: right factors B(L_tau, p_j)^T for j = J .. 0 from the current fields,
        one chunk at a time from the top (the per-sweep right stack)."""
        m, pts = self.m, self.m.points()
        J = len(pts) - 1
        for k, sigma in enumerate((+1, -1)):
            st.right[k] = {J: m.identity_udt()}
            for j in range(J - 1, -1, -1):
                st.right[k][j] = m.right_chunk(st.right[k][j + 1], st.fields, pts[j], pts[j + 1], sigma)
        st.right_valid = True

    def _sweep_chain(self, st: ChainState):
        """Up sweep: for l = 1 .. L_tau wrap to G(l), attempt slice l, stabilise at l = k n_s and
        l = L_tau.  Down sweep (odd global sweeps when sweep_mode bit 0 is set): for l = L_tau ..
        1 attempt slice l with G(l), unwrap to G(l-1), stabilise at l - 1 = k n_s (including 0).
        Either way the chain ends at G(0) = G(L_tau).

        Baseline mode keeps the factors the stabilisations need: an up sweep uses the right
        factors of the fields it has not visited yet (built at its start, or left by the down
        sweep before it) and pushes the slices it has visited onto the left factors; a down
        sweep does the same the other way round, with the left factors of the up sweep before."""
        m = self.m
        Lt = m.n_slices
        Gs = [st.G[0], st.G[1]]
        logdet_run = list(st.logdet)
        down = bool(m.sweep_mode & 1) and (st.sweeps_done % 2 == 1)
        pts = m.points()
        if not down:
            if m.stacks:
                if not ((m.sweep_mode & 1) and st.right_valid):
                    self._build_right(st)
                st.left = [{0: m.identity_udt()}, {0: m.identity_udt()}]
            for l in range(1, Lt + 1):
                s_l = st.fields[l - 1]
                Gs = [m.wrap(Gs[0], s_l, +1), m.wrap(Gs[1], s_l, -1)]
                self._metropolis_slice(st, Gs[0], Gs[1], l, logdet_run)
                if l % m.stab_every == 0 or l == Lt:
                    if m.stacks:
                        j = pts.index(l)
                        for k, sigma in enumerate((+1, -1)):
                            st.left[k][j] = m.left_chunk(st.left[k][j - 1], st.fields, pts[j - 1], l, sigma)
                    self._stabilise(st, Gs, l, logdet_run)
            st.right_valid = False
        else:
            if m.stacks:
                J = len(pts) - 1
                st.right = [{J: m.identity_udt()}, {J: m.identity_udt()}]
            for l in range(Lt, 0, -1):
                self._metropolis_slice(st, Gs[0], Gs[1], l, logdet_run)
                s_l = st.fields[l - 1]
                Gs = [m.unwrap(Gs[0], s_l, +1), m.unwrap(Gs[1], s_l, -1)]
                if (l - 1) % m.stab_every == 0:
                    if m.stacks:
                        j = pts.index(l - 1)
                        for k, sigma in enumerate((+1, -1)):
                            st.right[k][j] = m.right_chunk(st.right[k][j + 1], st.fields, l - 1,
                                                           pts[j + 1], sigma)
                    self._stabilise(st, Gs, l - 1, logdet_run)
            st.right_valid = True
        st.G = Gs
        st.logdet = logdet_run
        st.sweeps_done += 1

    def sweep(self, n_sweeps: int = 1, chains: Optional[List[int]] = None):
        for c in (range(len(self.chains)) if chains is None else chains):
            for _ in range(n_sweeps):
                self._sweep_chain(self.chains[c])

    def measure(self, stagger=None):
        """Per-chain observables from G(0) after the last sweep (one dict per chain); with a form
        factor `stagger` (+-1 per site) also the staggered spin structure factor."""
        out = []
        for st in self.chains:
            docc, dens, kin = measure_from_green(self.m.T, st.G[0], st.G[1])
            saf = spin_structure(st.G[0], st.G[1], stagger) if stagger is not None else None
            out.append(dict(double_occ=docc, density=dens, kinetic=kin, spin_af=saf,
                            logdet_up=st.logdet[0], logdet_dn=st.logdet[1],
                            max_drift=st.max_drift, max_logdet_err=st.max_logdet_err,
                            attempted=st.attempted, accepted=st.accepted,
                            near_ties=st.near_ties, flags=st.flags,
                            slice_double_occ=st.slice_docc / st.slice_meas if st.slice_meas else 0.0,
                            slice_kinetic=st.slice_kin / st.slice_meas if st.slice_meas else 0.0,
                            slice_meas=st.slice_meas))
        return out

    def fields(self) -> np.ndarray:
        return np.stack([st.fields for st in self.chains])

    def green(self) -> np.ndarray:
        """[n_chains][2][N][N] current G(0) of both spins."""
        return np.stack([np.stack(st.G) for st in self.chains])

    # -- fixed-field probes (no acceptance, no state change) -----------------------------
    def debug_green(self, l: int, n_wraps: int) -> np.ndarray:
        """Fresh G(l) of the current fields, then wrapped through slices l+1 .. l+n_wraps, or
        for n_wraps < 0 unwrapped through slices l, l-1, .. l+n_wraps+1 (G(l-1) = B_l^-1 G B_l)."""
        out = []
        for st in self.chains:
            per = []
            for sigma in (+1, -1):
                G, _ = self.m.green(st.fields, l, sigma)
                for w in range(1, n_wraps + 1):
                    G = self.m.wrap(G, st.fields[l + w - 1], sigma)
                for w in range(0, -n_wraps):
                    G = self.m.unwrap(G, st.fields[l - w - 1], sigma)
                per.append(G)
            out.append(np.stack(per))
        return np.stack(out)

    def debug_ratios(self, l: int) -> np.ndarray:
        """[n_chains][2][N]: R^up_i, R^dn_i for flipping s_{i,l} alone, from fresh G(l)."""
        out = []
        for st in self.chains:
            G_up, _ = self.m.green(st.fields, l, +1)
            G_dn, _ = self.m.green(st.fields, l, -1)
            r_up, r_dn = self.m.ratios(G_up, G_dn, st.fields[l - 1])
            out.append(np.stack([r_up, r_dn]))
        return np.stack(out)
