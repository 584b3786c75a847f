"""Exact references that pin the oracle: none of them runs the oracle's algorithm.

* Fock-space Trotter trace: the many-body operator exp(-dtau H_U) exp(-dtau H_k) of eq. (3)
  built on the full 4^N-dimensional Fock space (Jordan-Wigner), multiplied L_tau times and traced.
* Brute-force enumeration of all 2^(N L_tau) HS fields with plain determinants and inverses
  (no stabilisation: only for small beta, where I + B is well conditioned).
* Closed forms: U = 0 (free fermions) and the uniform field s = +1 everywhere, both from the
  eigendecomposition of T alone.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.linalg as sla


# ----------------------------------------------------------------------- Fock space
def fock_operators(n_modes: int):
    """Annihilators c_m (dense 2^n x 2^n) with Jordan-Wigner strings."""
    a = np.array([[0.0, 1.0], [0.0, 0.0]])       # |0><1| on one mode
    z = np.diag([1.0, -1.0])
    eye = np.eye(2)
    ops = []
    for m in range(n_modes):
        mats = [z] * m + [a] + [eye] * (n_modes - m - 1)
        op = mats[0]
        for M in mats[1:]:
            op = np.kron(op, M)
        ops.append(op)
    return ops


def fock_trotter(T: np.ndarray, U: float, dtau: float, n_slices: int, form=None):
    """Z and <O> at the slice boundary for the Trotterised Hubbard model of eq. (3).

    Modes: (i, up) -> i, (i, dn) -> N + i.  Returns Z = Tr[(e^{-dtau H_U} e^{-dtau H_k})^L],
    double occupancy per site and kinetic energy per site, both inserted at the right end; with a
    real form factor f also (1/N) <(sum_i f_i s^z_i)^2>, s^z_i = (n_i,up - n_i,dn)/2.
    """
    N = T.shape[0]
    c = fock_operators(2 * N)
    cd = [op.T for op in c]
    n = [cd[m] @ c[m] for m in range(2 * N)]
    dim = c[0].shape[0]
    I = np.eye(dim)
    Hk = np.zeros((dim, dim))
    for s in range(2):
        for i in range(N):
            for j in range(N):
                if T[i, j] != 0.0:
                    Hk += T[i, j] * cd[s * N + i] @ c[s * N + j]
    Hu = np.zeros((dim, dim))
    for i in range(N):
        Hu += U * (n[i] - 0.5 * I) @ (n[N + i] - 0.5 * I)
    # H_U is diagonal in the occupation basis
    slice_op = np.diag(np.exp(-dtau * np.diag(Hu))) @ sla.expm(-dtau * Hk)
    P = np.linalg.matrix_power(slice_op, n_slices)
    Z = float(np.trace(P))
    D = sum(n[i] @ n[N + i] for i in range(N)) / N
    docc = float(np.trace(P @ D)) / Z
    ekin = float(np.trace(P @ Hk)) / Z / N
    if form is None:
        return Z, docc, ekin
    Mz = sum(form[i] * 0.5 * (n[i] - n[N + i]) for i in range(N))
    return Z, docc, ekin, float(np.trace(P @ Mz @ Mz)) / Z / N


# ----------------------------------------------------------------------- enumeration
def _prop(T, dtau):
    lam, V = np.linalg.eigh(T)
    return (V * np.exp(-dtau * lam)) @ V.T


def enumerate_fields(T: np.ndarray, U: float, dtau: float, n_slices: int):
    """All HS fields: weights prod_sigma det(I + B^sigma(L,0)) and G(0) of both spins.

    Returns (fields [n_cfg][L][N], weights [n_cfg], G_up [n_cfg][N][N], G_dn) with plain
    (unstabilised) products, determinants and inverses.
    """
    N = T.shape[0]
    nu = math.acosh(math.exp(0.5 * U * dtau))
    K = _prop(T, dtau)
    n_cfg = 2 ** (N * n_slices)
    bits = ((np.arange(n_cfg)[:, None] >> np.arange(N * n_slices)[None, :]) & 1)
    fields = (2 * bits - 1).reshape(n_cfg, n_slices, N).astype(np.float64)
    out_w = np.ones(n_cfg)
    Gs = []
    for sigma in (+1, -1):
        B = np.broadcast_to(np.eye(N), (n_cfg, N, N)).copy()
        for l in range(n_slices):
            Bl = np.exp(sigma * nu * fields[:, l, :])[:, :, None] * K[None]
            B = Bl @ B
        M = np.eye(N)[None] + B
        out_w *= np.linalg.det(M)
        Gs.append(np.linalg.inv(M))
    return fields, out_w, Gs[0], Gs[1]


def enumerate_observables(T: np.ndarray, U: float, dtau: float, n_slices: int):
    """Exact Trotterised <double occupancy>, <E_k per site>, Z from the HS sum."""
    N = T.shape[0]
    fields, w, Gu, Gd = enumerate_fields(T, U, dtau, n_slices)
    gu = np.diagonal(Gu, axis1=1, axis2=2)
    gd = np.diagonal(Gd, axis1=1, axis2=2)
    docc = np.sum((1 - gu) * (1 - gd), axis=1) / N
    eye = np.eye(N)
    ek = (np.einsum("ij,cji->c", T, eye[None] - Gu) + np.einsum("ij,cji->c", T, eye[None] - Gd)) / N
    Z = (0.5 * math.exp(-0.25 * U * dtau)) ** (N * n_slices) * np.sum(w)
    return float(Z), float(np.sum(w * docc) / np.sum(w)), float(np.sum(w * ek) / np.sum(w))


# ----------------------------------------------------------------------- closed forms
def free_green(T: np.ndarray, beta: float) -> np.ndarray:
    """U = 0: G = (I + e^{-beta T})^{-1} = V Diag(1 / (1 + e^{-beta lambda})) V^T."""
    lam, V = np.linalg.eigh(T)
    return (V * (1.0 / (1.0 + np.exp(-beta * lam)))) @ V.T


def free_kinetic(T: np.ndarray, beta: float) -> float:
    """U = 0 kinetic energy per site: (2/N) sum_k lambda_k f(lambda_k), f = 1/(1 + e^{beta lambda})."""
    lam = np.linalg.eigvalsh(T)
    return float(2.0 * np.sum(lam / (1.0 + np.exp(beta * lam))) / T.shape[0])


def uniform_field_green(T: np.ndarray, nu: float, n_slices: int, beta: float, sigma: int):
    """s = +1 everywhere: B(beta,0) = e^{sigma nu L} e^{-beta T}, G = V Diag(1/(1+e^{sigma nu L - beta lambda})) V^T."""
    lam, V = np.linalg.eigh(T)
    x = sigma * nu * n_slices - beta * lam
    return (V * (1.0 / (1.0 + np.exp(x)))) @ V.T


def all_occupation_states():
    return list(itertools.product((0, 1), repeat=2))
