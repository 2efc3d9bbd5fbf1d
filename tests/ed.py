"""Exact diagonalisation references for the oracle pins.

The dense Hamiltonian here is assembled independently of the oracle: block
basis [all electron components; all hole components] (the oracle interleaves),
the hopping matrix from Kronecker products of 1D adjacency matrices, and the
Nambu structure H = [[h, P], [conj(P), -conj(h)]] of eq. (hamil2) with
h = -t A + diag(eps - mu) and P the (symmetric) pairing matrix.
"""
from __future__ import annotations

import numpy as np


def adjacency_1d(L: int, periodic: bool) -> np.ndarray:
    A = np.zeros((L, L))
    for i in range(L - 1):
        A[i, i + 1] = A[i + 1, i] = 1.0
    if periodic and L >= 3:
        A[0, L - 1] = A[L - 1, 0] = 1.0
    return A


def normal_block(w, use_phases=True) -> np.ndarray:
    """h = -t_ij hopping + diag(eps - mu), with Peierls phases when present."""
    Lx, Ly = w.Lx, w.Ly
    if w.peierls is None or not use_phases:
        A = np.kron(np.eye(Ly), adjacency_1d(Lx, w.bc_x == 1)) + \
            np.kron(adjacency_1d(Ly, w.bc_y == 1), np.eye(Lx))
        h = -w.t * A.astype(np.complex128)
    else:
        h = np.zeros((Lx * Ly, Lx * Ly), dtype=np.complex128)
        for y in range(Ly):
            for x in range(Lx):
                s = x + Lx * y
                for axis, (dx, dy) in enumerate(((1, 0), (0, 1))):
                    jx, jy = x + dx, y + dy
                    if jx >= Lx:
                        if w.bc_x != 1:
                            continue
                        jx -= Lx
                    if jy >= Ly:
                        if w.bc_y != 1:
                            continue
                        jy -= Ly
                    j = jx + Lx * jy
                    tij = w.t * np.exp(1j * w.peierls[axis][s])
                    h[s, j] += -tij
                    h[j, s] += -np.conj(tij)
    h += np.diag(w.eps - w.mu_c)
    return h


def pairing_block(w, delta) -> np.ndarray:
    Lx, Ly = w.Lx, w.Ly
    P = np.diag(np.asarray(delta, dtype=np.complex128))
    if w.delta_bond is not None:
        for y in range(Ly):
            for x in range(Lx):
                s = x + Lx * y
                for axis, (dx, dy) in enumerate(((1, 0), (0, 1))):
                    jx, jy = x + dx, y + dy
                    if jx >= Lx:
                        if w.bc_x != 1:
                            continue
                        jx -= Lx
                    if jy >= Ly:
                        if w.bc_y != 1:
                            continue
                        jy -= Ly
                    j = jx + Lx * jy
                    P[s, j] += w.delta_bond[axis][s]
                    P[j, s] += w.delta_bond[axis][s]
    return P


def dense_H(w, delta=None) -> np.ndarray:
    h = normal_block(w)
    P = pairing_block(w, w.delta if delta is None else delta)
    return np.block([[h, P], [np.conj(P), -np.conj(h)]])


def eig(w, a, b, delta=None):
    H = dense_H(w, delta)
    if np.max(np.abs(H.imag)) == 0.0:
        H = H.real          # real symmetric: real eigenvectors
    E, V = np.linalg.eigh(H)
    return (E - b) / a, V


def cheb_T(n, x):
    return np.cos(np.multiply.outer(np.asarray(n, dtype=float), np.arccos(np.clip(x, -1, 1))))


def ed_moments(w, a, b, sites, N, delta=None):
    """mu_ee_n(i) = sum_k |u_k(i)|^2 T_n(E_k), mu_he_n(i) = sum_k v_k(i) conj(u_k(i)) T_n(E_k)
    (Lehmann form eq. (imag1) with the moments of eqs. (coeff1)/(coeff2))."""
    Et, V = eig(w, a, b, delta)
    L2 = w.L2
    T = cheb_T(np.arange(N), Et)                   # [N, D]
    sites = np.asarray(sites)
    u = V[sites, :]
    v = V[L2 + sites, :]
    mu_ee = (np.abs(u) ** 2) @ T.T
    mu_he = (v * np.conj(u)) @ T.T
    return mu_ee, mu_he


def cheb_divided_difference(n, x, y):
    """(T_n(x) - T_n(y)) / (x - y) with its limit n U_{n-1}(x) at x = y,
    written through x = cos(al), y = cos(be) so it stays stable."""
    al = np.arccos(np.clip(x, -1, 1))
    be = np.arccos(np.clip(y, -1, 1))
    n = np.asarray(n, dtype=float)[..., None, None]
    sp = np.sin((al + be) / 2)
    sm = np.sin((al - be) / 2)
    close = np.abs(al - be) < 1e-7
    sm_safe = np.where(close, 1.0, sm)
    gen = np.sin(n * (al + be) / 2) * np.sin(n * (al - be) / 2) / (sp * sm_safe)
    lim = n * np.sin(n * al) / np.sin(al)
    return np.where(close, lim, gen)
