"""Seeded synthetic lattices for the Chebyshev-BdG hot path.

This module only *describes inputs*: lattice sizes, the on-site potential
landscape, the initial order parameter, bond pairing and vector-potential
phases, the start sites and the energy grid.  It holds none of the method's
arithmetic (no Hamiltonian, no rescaling, no moments, no kernels), so both the
CPU oracle and the GPU path can draw from it without sharing any computation.

Site index convention: s = x + Lx * y (x fastest).
Bond arrays have shape [2, L2]: row 0 is the bond s -> s + x^, row 1 is
s -> s + y^.  A bond that leaves an open lattice is stored as 0 and ignored.

The workloads follow the paper's model Hamiltonian, eq. (hamil2): nearest
neighbour hopping t, on-site potential eps_i (impurities), chemical potential
mu, on-site pairing Delta_i or bond pairing Delta_ij, and Peierls phases of a
perpendicular field (the paragraph after eq. (hamil2)).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

OPEN = 0
PERIODIC = 1


@dataclass
class Workload:
    name: str
    Lx: int
    Ly: int
    bc_x: int
    bc_y: int
    t: float
    mu_c: float            # chemical potential (the paper's mu)
    U: float               # attractive on-site coupling (0: not self-consistent)
    eps: np.ndarray        # [L2] float64 on-site potential eps_i
    delta: np.ndarray      # [L2] float64 or complex128 initial on-site Delta_i
    delta_bond: Optional[np.ndarray]  # [2, L2] complex128 bond Delta_ij or None
    peierls: Optional[np.ndarray]     # [2, L2] float64 bond phases theta_ij or None
    N: int                 # number of Chebyshev moments, n = 0..N-1
    start_sites: np.ndarray  # int32 start sites |s,e>
    tile: int              # start vectors per tile
    energies: Optional[np.ndarray] = None  # float64 LDOS energies (units of t)
    kernel: str = "jackson"
    eta: float = 0.01      # spectral safety margin of the rescaling
    scalar: str = "real"   # "real" or "complex"
    pairing: str = "onsite"  # "onsite" or "bond"
    notes: dict = field(default_factory=dict)

    @property
    def L2(self) -> int:
        return self.Lx * self.Ly

    @property
    def D(self) -> int:
        return 2 * self.Lx * self.Ly

    @property
    def delta_cap(self) -> float:
        # every gap-map iterate satisfies |Delta| <= U/2, so the spectral bound
        # is taken with |Delta_i| raised to at least U/2 (fixed for the whole SCF)
        return 0.5 * self.U

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def site(Lx: int, x: int, y: int) -> int:
    return x + Lx * y


def _uniform_delta(L2: int, value: float) -> np.ndarray:
    return np.full(L2, value, dtype=np.float64)


def config0() -> Workload:
    """16x16 open lattice, one impurity V=5 at the centre site (8,8)."""
    Lx = Ly = 16
    eps = np.zeros(Lx * Ly)
    eps[site(Lx, 8, 8)] = 5.0
    return Workload(
        name="cfg0_16x16_N256_fp64", Lx=Lx, Ly=Ly, bc_x=OPEN, bc_y=OPEN,
        t=1.0, mu_c=-0.5, U=2.0, eps=eps, delta=_uniform_delta(Lx * Ly, 0.1),
        delta_bond=None, peierls=None, N=256,
        start_sites=np.arange(Lx * Ly, dtype=np.int32), tile=256)


def disorder(L2: int, frac: float, lo: float, hi: float, seed: int) -> np.ndarray:
    """round(frac*L2) distinct sites drawn without replacement, then V~U[lo,hi]."""
    rng = np.random.default_rng(seed)
    n_imp = int(round(frac * L2))
    where = rng.choice(L2, n_imp, replace=False)
    vals = rng.uniform(lo, hi, n_imp)
    eps = np.zeros(L2)
    eps[where] = vals
    return eps


def impurities(L2: int, count: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    where = rng.choice(L2, count, replace=False)
    vals = rng.uniform(lo, hi, count)
    eps = np.zeros(L2)
    eps[where] = vals
    return eps


def config1(L: int = 256, N: int = 1024, tile: int = 1024) -> Workload:
    """256x256 open lattice, 1% of sites disordered with V~U[-2,2] (seed 1)."""
    L2 = L * L
    return Workload(
        name=f"cfg1_{L}x{L}_N{N}_fp64", Lx=L, Ly=L, bc_x=OPEN, bc_y=OPEN,
        t=1.0, mu_c=-0.4, U=2.5, eps=disorder(L2, 0.01, -2.0, 2.0, seed=1),
        delta=_uniform_delta(L2, 0.1), delta_bond=None, peierls=None, N=N,
        start_sites=np.arange(L2, dtype=np.int32), tile=tile)


def config2(L: int = 256, N: int = 2048, tile: int = 1024) -> Workload:
    """The config-1 lattice with N=2048 moments, for the FP32 recursion."""
    w = config1(L, N, tile)
    return w.with_(name=f"cfg2_{L}x{L}_N{N}_fp32")


def landau_phases(Lx: int, Ly: int, f: float) -> np.ndarray:
    """Bond phases of a uniform perpendicular field in the Landau gauge.

    theta on the +x bond leaving (x, y) is -pi*f*y, and 0 on +y bonds, so the
    phase collected anticlockwise around every plaquette is pi*f, i.e. a flux
    f*phi0 with phi0 = h/2e (Peierls substitution of eq. (hamil2)).
    """
    y = np.repeat(np.arange(Ly), Lx).astype(np.float64)
    th = np.zeros((2, Lx * Ly))
    th[0] = -np.pi * f * y
    return th


def vortex_dwave_bonds(Lx: int, Ly: int, amp: float, centres, heal: float = 4.0,
                       bc_x: int = OPEN, bc_y: int = OPEN) -> np.ndarray:
    """Synthetic d-wave bond pairing with phase windings around given points.

    Delta on the +x bond is +amp, on the +y bond -amp (d_{x^2-y^2} symmetry),
    each multiplied by prod_v tanh(rho_v/heal) exp(i phi_v), where (rho_v, phi_v)
    are the polar coordinates of the bond midpoint seen from centre v.  This is
    a fixed input profile, not a self-consistent solution.
    """
    xs = np.tile(np.arange(Lx), Ly).astype(np.float64)
    ys = np.repeat(np.arange(Ly), Lx).astype(np.float64)
    out = np.zeros((2, Lx * Ly), dtype=np.complex128)
    for d, (mx, my, sign) in enumerate(((0.5, 0.0, 1.0), (0.0, 0.5, -1.0))):
        px, py = xs + mx, ys + my
        prof = np.ones(Lx * Ly, dtype=np.complex128)
        for (cx, cy) in centres:
            dx, dy = px - cx, py - cy
            rho = np.hypot(dx, dy)
            prof *= np.tanh(rho / heal) * np.exp(1j * np.arctan2(dy, dx))
        out[d] = sign * amp * prof
    if bc_x == OPEN:
        out[0][xs == Lx - 1] = 0.0
    if bc_y == OPEN:
        out[1][ys == Ly - 1] = 0.0
    return out


def config3(L: int = 512, N: int = 2048, stride: int = 8, n_e: int = 512,
            tile: int = 1024, f: float = 1.0 / 256.0) -> Workload:
    """512x512 open lattice, Peierls flux f per plaquette, d-wave bond pairing
    with four phase windings, LDOS at 512 energies on a stride-8 site grid."""
    q = L // 4
    centres = [(q - 0.5, q - 0.5), (3 * q - 0.5, q - 0.5),
               (q - 0.5, 3 * q - 0.5), (3 * q - 0.5, 3 * q - 0.5)]
    off = stride // 2
    g = np.arange(off, L, stride)
    sites = (g[None, :] + L * g[:, None]).reshape(-1).astype(np.int32)
    energies = -2.0 + 4.0 * np.arange(n_e) / (n_e - 1)
    return Workload(
        name=f"cfg3_{L}x{L}_N{N}_c128", Lx=L, Ly=L, bc_x=OPEN, bc_y=OPEN,
        t=1.0, mu_c=-0.4, U=0.0, eps=np.zeros(L * L),
        delta=np.zeros(L * L, dtype=np.complex128),
        delta_bond=vortex_dwave_bonds(L, L, 0.1, centres),
        peierls=landau_phases(L, L, f), N=N, start_sites=sites, tile=tile,
        energies=energies, scalar="complex", pairing="bond",
        notes={"flux_per_plaquette_phi0": f, "vortex_centres": centres,
               "self_consistent": False})


def config4(L: int = 128, N: int = 512, tile: int = 1024) -> Workload:
    """128x128 open lattice, 64 impurities V~U[0,4] (seed 4), for gradients."""
    L2 = L * L
    return Workload(
        name=f"cfg4_{L}x{L}_N{N}_fp64", Lx=L, Ly=L, bc_x=OPEN, bc_y=OPEN,
        t=1.0, mu_c=-0.5, U=2.0, eps=impurities(L2, 64 if L == 128 else max(1, L2 // 256), 0.0, 4.0, seed=4),
        delta=_uniform_delta(L2, 0.1), delta_bond=None, peierls=None, N=N,
        start_sites=np.arange(L2, dtype=np.int32), tile=tile,
        notes={"centre_site": site(L, L // 2, L // 2)})


def small_random(Lx: int, Ly: int, N: int, seed: int, *, bc_x: int = OPEN,
                 bc_y: int = OPEN, complex_: bool = False, bond: bool = False,
                 flux: float = 0.0, n_sites: Optional[int] = None,
                 U: float = 2.0) -> Workload:
    """A small irregular case for parity tests: random potential and gap."""
    rng = np.random.default_rng(seed)
    L2 = Lx * Ly
    eps = rng.uniform(-1.5, 1.5, L2)
    if complex_:
        delta = rng.uniform(0.0, 0.3, L2) * np.exp(1j * rng.uniform(-np.pi, np.pi, L2))
    else:
        delta = rng.uniform(0.0, 0.3, L2)
    dbond = None
    if bond:
        dbond = (rng.uniform(-0.2, 0.2, (2, L2))
                 + (1j * rng.uniform(-0.2, 0.2, (2, L2)) if complex_ else 0.0)).astype(np.complex128)
        xs = np.tile(np.arange(Lx), Ly)
        ys = np.repeat(np.arange(Ly), Lx)
        if bc_x == OPEN:
            dbond[0][xs == Lx - 1] = 0.0
        if bc_y == OPEN:
            dbond[1][ys == Ly - 1] = 0.0
    ph = landau_phases(Lx, Ly, flux) if (complex_ and flux != 0.0) else None
    if n_sites is None:
        sites = np.arange(L2, dtype=np.int32)
    else:
        sites = np.sort(rng.choice(L2, n_sites, replace=False)).astype(np.int32)
    return Workload(
        name=f"rand_{Lx}x{Ly}_N{N}_s{seed}", Lx=Lx, Ly=Ly, bc_x=bc_x, bc_y=bc_y,
        t=1.0, mu_c=rng.uniform(-0.8, 0.2), U=U, eps=eps, delta=delta,
        delta_bond=dbond, peierls=ph, N=N, start_sites=sites, tile=len(sites),
        scalar="complex" if complex_ else "real",
        pairing="bond" if bond else "onsite")


def sn_surface(Lx_n: int = 380, Lx_s: int = 20, Ly: int = 500, N: int = 2000, delta: float = 0.1,
               mu_c: float = -0.4, n_sites: int = 64) -> Workload:
    """The planar normal-metal / s-wave superconductor system of the first
    example (its text: L_x^N = 380a, L_x^S = 20a, L_y = 500a, Delta = 0.1t;
    the caption's 300/20 swaps the regions): normal metal on x < Lx_n with a
    free surface at x = 0, superconductor on x >= Lx_n, periodic in y (the
    planar geometry).  Delta is fixed (not self-consistent); the start sites
    are n_sites consecutive surface sites x = 0 around y = Ly/2.  The example
    gives no chemical potential: mu_c = -0.4 as in the other workloads."""
    Lx = Lx_n + Lx_s
    L2 = Lx * Ly
    xs = np.tile(np.arange(Lx), Ly)
    d = np.where(xs >= Lx_n, delta, 0.0)
    y0 = Ly // 2 - n_sites // 2
    sites = np.array([site(Lx, 0, y0 + k) for k in range(n_sites)], dtype=np.int32)
    return Workload(name=f"sn_surface_{Lx_n}+{Lx_s}x{Ly}_N{N}", Lx=Lx, Ly=Ly, bc_x=OPEN, bc_y=PERIODIC,
                    t=1.0, mu_c=mu_c, U=0.0, eps=np.zeros(L2), delta=d, delta_bond=None, peierls=None,
                    N=N, start_sites=sites, tile=n_sites, energies=np.linspace(-0.2, 0.2, 401),
                    kernel="lorentz", notes={"broadening": 0.001, "surface_x": 0})


def sns_impurity(N: int = 2048, V: float = 2.0, delta: float = 0.1, mu_c: float = -0.4,
                 superconducting: bool = True, impurity: bool = True, window: int = 10) -> Workload:
    """The SC / normal metal / SC sandwich of the second example, 50a/50a/50a x
    100a (superconductor on x < 50 and x >= 100), with the Gaussian impurity
    V_i = V exp(-|r_i - r_0|^2 / a^2), V = 2t, r_0 = (60a, 50a) in the normal
    layer; superconducting=False gives the homogeneous normal metal of the
    comparison panels, impurity=False the clean system whose LDOS is
    subtracted.  The example gives neither Delta nor mu: Delta = 0.1t as in
    the first example, mu_c = -0.4.  Open boundaries; fixed Delta.  Start
    sites: the (2 window + 1)^2 square around r_0."""
    Lx, Ly = 150, 100
    L2 = Lx * Ly
    xs, ys = np.tile(np.arange(Lx), Ly), np.repeat(np.arange(Ly), Lx)
    d = np.where((xs < 50) | (xs >= 100), delta, 0.0) if superconducting else np.zeros(L2)
    eps = V * np.exp(-((xs - 60.0) ** 2 + (ys - 50.0) ** 2)) if impurity else np.zeros(L2)
    sites = np.array([site(Lx, 60 + dx, 50 + dy) for dy in range(-window, window + 1)
                      for dx in range(-window, window + 1)], dtype=np.int32)
    tag = ("sns" if superconducting else "normal") + ("_imp" if impurity else "_clean")
    return Workload(name=f"{tag}_150x100_N{N}", Lx=Lx, Ly=Ly, bc_x=OPEN, bc_y=OPEN, t=1.0, mu_c=mu_c, U=0.0,
                    eps=eps, delta=d, delta_bond=None, peierls=None, N=N, start_sites=sites,
                    tile=len(sites), energies=np.array([0.0, 0.03, 0.06]),
                    notes={"impurity_centre": (60, 50), "window": window})


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}
