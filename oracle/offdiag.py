"""Off-diagonal moments between a start site and its four lattice neighbours,
the bond order parameter and the bond current (test infrastructure, FP64).

The moments of the paragraph after eq. (ref2) with a bra on another grid
point: mu^{ee}_n(j; i) = <j,e|T_n(Ht)|i,e>, mu^{he}_n(j; i) = <j,h|T_n(Ht)|i,e>,
read off the same vector recursion a_n = T_n(Ht)|i,e> at the sites j next to
i.  Neighbour order: +x, -x, +y, -y (a missing neighbour of an open lattice
gives zero rows).
"""
from __future__ import annotations

import numpy as np

NEIGHBOURS = ((1, 0), (-1, 0), (0, 1), (0, -1))


def neighbour_site(Lx, Ly, bc_x, bc_y, s, d):
    """Site index of neighbour d of site s, or -1 outside an open lattice."""
    x, y = s % Lx, s // Lx
    dx, dy = NEIGHBOURS[d]
    x2, y2 = x + dx, y + dy
    if not 0 <= x2 < Lx:
        if not bc_x:
            return -1
        x2 %= Lx
    if not 0 <= y2 < Ly:
        if not bc_y:
            return -1
        y2 %= Ly
    return x2 + Lx * y2


def neighbour_moments(H, Lx, Ly, bc_x, bc_y, sites, N):
    """nb_ee[k, d, n] = <j,e|a_n>, nb_he[k, d, n] = <j,h|a_n> with
    a_n = T_n(Ht)|s_k,e> by the recursion of eq. (ref2) (a plain sparse
    matrix-vector product per step), j = neighbour d of s_k."""
    A = H.to_scipy()
    D = A.shape[0]
    sites = np.asarray(sites)
    ee = np.zeros((len(sites), 4, N), dtype=np.complex128)
    he = np.zeros((len(sites), 4, N), dtype=np.complex128)
    for k, s in enumerate(sites):
        js = [neighbour_site(Lx, Ly, bc_x, bc_y, int(s), d) for d in range(4)]
        prev = np.zeros(D, dtype=np.complex128)
        prev[2 * s] = 1.0
        cur = A @ prev
        for n in range(N):
            a = prev if n == 0 else cur
            for d, j in enumerate(js):
                if j >= 0:
                    ee[k, d, n] = a[2 * j]
                    he[k, d, n] = a[2 * j + 1]
            if n >= 1:
                prev, cur = cur, 2.0 * (A @ cur) - prev
    return ee, he


def bond_gap_map(nb_he, U, Lx, Ly, bc_x, bc_y, weights):
    """Bond order parameter of eq. (op1) for i != j, symmetrised (singlet):
    Delta_ij = (U/4) [conj(<j,h|w(Ht)|i,e>) + conj(<i,h|w(Ht)|j,e>)], with
    w(Ht) ~ sum_n weights_n T_n(Ht) (weights = g_n c_n of the gap weight).
    Rows of nb_he are indexed by site (all L2 sites).  Returns [2, L2]: the
    +x and +y bond of every site, 0 where the bond leaves an open lattice."""
    S = np.asarray(nb_he) @ np.asarray(weights)         # [L2, 4]
    L2 = Lx * Ly
    out = np.zeros((2, L2), dtype=np.complex128)
    for s in range(L2):
        for axis, (fwd, back) in enumerate(((0, 1), (2, 3))):
            j = neighbour_site(Lx, Ly, bc_x, bc_y, s, fwd)
            if j >= 0:
                out[axis, s] = 0.25 * U * (np.conj(S[s, fwd]) + np.conj(S[j, back]))
    return out


def bond_current(nb_ee, t, peierls, Lx, Ly, bc_x, bc_y, weights):
    """Particle current along the +x and +y bond of every site, both spins:
    J_{i->j} = 4 Im(t_ij <c_i^+ c_j>) for the hopping -t_ij c_i^+ c_j of
    eq. (hamil2) (t_ij = t exp(i theta_ij)), with
    <c_i^+ c_j> = <j,e| f(Ht) |i,e> ~ sum_n weights_n mu^{ee}_n(j; i)
    (weights = g_n c_n of f).  Reading of the printed current equation, whose
    imaginary part of a real quantity is garbled.  Returns [2, L2]."""
    rho = np.asarray(nb_ee) @ np.asarray(weights)        # [L2, 4]
    L2 = Lx * Ly
    out = np.zeros((2, L2))
    for s in range(L2):
        for axis, fwd in enumerate((0, 2)):
            j = neighbour_site(Lx, Ly, bc_x, bc_y, s, fwd)
            if j >= 0:
                th = 0.0 if peierls is None else peierls[axis][s]
                out[axis, s] = 4.0 * np.imag(t * np.exp(1j * th) * rho[s, fwd])
    return out
