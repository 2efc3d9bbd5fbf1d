"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check is an exact
diagonalisation, a closed form, an invariant, quadrature, or finite
differences, chosen so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""
import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads as W
from tests import ed


def _small(Lx=6, Ly=5, seed=3, **kw):
    return W.small_random(Lx, Ly, N=64, seed=seed, **kw)


# ---------------------------------------------------------------- P1: ED moments
@pytest.mark.parametrize("case", [
    dict(),
    dict(bc_x=W.PERIODIC, bc_y=W.PERIODIC),
    dict(bc_x=W.PERIODIC),
    dict(complex_=True),
    dict(complex_=True, bond=True, flux=0.25),
    dict(bond=True),
])
def test_moments_equal_exact_diagonalisation(case):
    w = _small(**case)
    e0, e1, a, b = oracle.workload_bounds(w)
    mu_ee, mu_he = oracle.workload_moments(w, a, b, N=96)
    r_ee, r_he = ed.ed_moments(w, a, b, w.start_sites, 96)
    assert np.max(np.abs(mu_ee - r_ee.real)) < 1e-12
    assert np.max(np.abs(r_ee.imag)) < 1e-12
    assert np.max(np.abs(mu_he - r_he)) < 1e-12


def test_config0_moments_equal_exact_diagonalisation():
    w = W.config0()
    _, _, a, b = oracle.workload_bounds(w)
    assert abs(a - 2 * 10.5 / 1.99) < 1e-12      # Gershgorin: |5+0.5| + U/2 + 4t
    mu_ee, mu_he = oracle.workload_moments(w, a, b)
    r_ee, r_he = ed.ed_moments(w, a, b, w.start_sites, w.N)
    assert np.max(np.abs(mu_ee - r_ee.real)) < 1e-12
    assert np.max(np.abs(mu_he - r_he.real)) < 1e-12


def test_nonzero_b_shift_equals_exact_diagonalisation():
    # an asymmetric interval exercises the -b/a diagonal shift
    w = _small(seed=11)
    a, b = 6.5, 0.37
    mu_ee, mu_he = oracle.workload_moments(w, a, b, N=50)
    r_ee, r_he = ed.ed_moments(w, a, b, w.start_sites, 50)
    assert np.max(np.abs(mu_ee - r_ee.real)) < 1e-12
    assert np.max(np.abs(mu_he - r_he.real)) < 1e-12


# ---------------------------------------------- P2: completeness and low moments
@pytest.mark.parametrize("complex_", [False, True])
def test_first_moments(complex_):
    w = _small(complex_=complex_, bond=True, flux=0.3 if complex_ else 0.0)
    a, b = 7.0, 0.0
    H = oracle.workload_csr(w, a, b)
    mu_ee, mu_he = oracle.moments(H, w.start_sites, 3)
    assert np.all(mu_ee[:, 0] == 1.0) and np.all(mu_he[:, 0] == 0.0)
    assert np.max(np.abs(mu_ee[:, 1] - (w.eps - w.mu_c - b) / a)) < 1e-15
    assert np.max(np.abs(mu_he[:, 1] - np.conj(w.delta) / a)) < 1e-15
    # mu_2 = 2 ||Ht e_{i,e}||^2 - 1, with the column norm from the dense ED matrix
    Hd = (ed.dense_H(w) - b * np.eye(w.D)) / a
    col = np.linalg.norm(Hd[:, :w.L2], axis=0) ** 2
    assert np.max(np.abs(mu_ee[:, 2] - (2 * col - 1))) < 1e-14


# ---------------------------------------------------------- P3: particle-hole symmetry
@pytest.mark.parametrize("case", [dict(), dict(complex_=True, bond=True, flux=0.2)])
def test_particle_hole_symmetry(case):
    w = _small(**case)
    _, _, a, b = oracle.workload_bounds(w)
    assert b == 0.0
    mu_ee, mu_he = oracle.workload_moments(w, a, b, N=80)
    # <i,h|T_n|i,e> vanishes for even n when H anticommutes with C(u,v) = (-v*, u*)
    assert np.max(np.abs(mu_he[:, 0::2])) < 1e-13
    # the spectrum is symmetric
    E = np.linalg.eigvalsh(ed.dense_H(w))
    assert np.max(np.abs(np.sort(E) + np.sort(E)[::-1])) < 1e-12


# ------------------------------------------------- P4: Bloch closed form (periodic)
@pytest.mark.parametrize("L,N", [(8, 64), (24, 200)])
def test_bloch_closed_form_periodic(L, N):
    t, mu, dl = 1.0, -0.3, 0.25
    w = W.Workload("bloch", L, L, W.PERIODIC, W.PERIODIC, t, mu, 0.0, np.zeros(L * L),
                   np.full(L * L, dl), None, None, N, np.array([0, L + 3, L * L - 1], np.int32), 3)
    a = 6.1
    mu_ee, mu_he = oracle.workload_moments(w, a, 0.0)
    k = 2 * np.pi * np.arange(L) / L
    xi = (-2 * t * (np.cos(k)[:, None] + np.cos(k)[None, :]) - mu).ravel()
    E = np.sqrt(xi ** 2 + dl ** 2)
    Tp, Tm = ed.cheb_T(np.arange(N), E / a), ed.cheb_T(np.arange(N), -E / a)
    u2, v2 = (1 + xi / E) / 2, (1 - xi / E) / 2
    ref_ee = (Tp @ u2 + Tm @ v2) / L ** 2
    ref_he = ((Tp - Tm) @ (dl / (2 * E))) / L ** 2
    assert np.max(np.abs(mu_ee - ref_ee[None, :])) < 1e-13
    assert np.max(np.abs(mu_he - ref_he[None, :])) < 1e-13


# ------------------------------------------- P5: open-boundary sine-mode closed form
def test_open_boundary_sine_modes():
    Lx, Ly, t, mu, dl, N = 9, 7, 1.0, 0.2, 0.15, 120
    sites = np.array([0, 4 + 9 * 3, 8 + 9 * 6, 2 + 9 * 1], np.int32)
    w = W.Workload("sine", Lx, Ly, W.OPEN, W.OPEN, t, mu, 0.0, np.zeros(Lx * Ly),
                   np.full(Lx * Ly, dl), None, None, N, sites, 4)
    a = 5.5
    mu_ee, mu_he = oracle.workload_moments(w, a, 0.0)

    def modes(L):
        m = np.arange(1, L + 1)
        x = np.arange(L)
        phi = np.sqrt(2 / (L + 1)) * np.sin(np.pi * np.outer(m, x + 1) / (L + 1))
        return -2 * t * np.cos(np.pi * m / (L + 1)), phi

    ex, px = modes(Lx)
    ey, py = modes(Ly)
    xi = (ex[:, None] + ey[None, :] - mu).ravel()
    E = np.sqrt(xi ** 2 + dl ** 2)
    Tp, Tm = ed.cheb_T(np.arange(N), E / a), ed.cheb_T(np.arange(N), -E / a)
    for q, s in enumerate(sites):
        x, y = s % Lx, s // Lx
        wgt = (px[:, x][:, None] ** 2 * py[:, y][None, :] ** 2).ravel()
        ref_ee = Tp @ (wgt * (1 + xi / E) / 2) + Tm @ (wgt * (1 - xi / E) / 2)
        ref_he = (Tp - Tm) @ (wgt * dl / (2 * E))
        assert np.max(np.abs(mu_ee[q] - ref_ee)) < 1e-13
        assert np.max(np.abs(mu_he[q] - ref_he)) < 1e-13


# ----------------------------------------------------------- P6: atomic limit t = 0
def test_atomic_limit():
    rng = np.random.default_rng(5)
    Lx, Ly, N = 5, 4, 100
    eps = rng.uniform(-2, 2, Lx * Ly)
    dl = rng.uniform(0.05, 0.5, Lx * Ly) * np.exp(1j * rng.uniform(-3, 3, Lx * Ly))
    w = W.Workload("atomic", Lx, Ly, W.OPEN, W.OPEN, 0.0, -0.4, 0.0, eps, dl, None, None, N,
                   np.arange(Lx * Ly, dtype=np.int32), Lx * Ly, scalar="complex")
    a = 4.0
    mu_ee, mu_he = oracle.workload_moments(w, a, 0.0)
    xi = eps + 0.4
    R = np.sqrt(xi ** 2 + np.abs(dl) ** 2)
    Tp, Tm = ed.cheb_T(np.arange(N), R / a).T, ed.cheb_T(np.arange(N), -R / a).T
    ref_ee = ((1 + xi / R)[:, None] * Tp + (1 - xi / R)[:, None] * Tm) / 2
    ref_he = (np.conj(dl) / (2 * R))[:, None] * (Tp - Tm)
    assert np.max(np.abs(mu_ee - ref_ee)) < 1e-13
    assert np.max(np.abs(mu_he - ref_he)) < 1e-13


# ------------------------------------------------------ Peierls phases (Hofstadter)
@pytest.mark.parametrize("L", [4, 6, 8])
def test_pi_flux_hofstadter_spectrum(L):
    """f = 1 puts a hopping phase pi on every plaquette; on an LxL torus the
    spectrum is then +-2t sqrt(cos^2 kx + cos^2 ky), ky over half the zone."""
    ph = W.landau_phases(L, L, 1.0)
    H = oracle.build_csr(L, L, 1, 1, 1.0, 0.0, np.zeros(L * L), np.zeros(L * L), None, ph)
    Hd = H.to_scipy().toarray()
    he, hh = Hd[0::2, 0::2], Hd[1::2, 1::2]
    k = 2 * np.pi * np.arange(L) / L
    kh = 2 * np.pi * np.arange(L // 2) / L
    e = 2 * np.sqrt(np.cos(k)[:, None] ** 2 + np.cos(kh)[None, :] ** 2).ravel()
    ref = np.sort(np.concatenate([e, -e]))
    assert np.max(np.abs(np.sort(np.linalg.eigvalsh(he)) - ref)) < 1e-12
    assert np.max(np.abs(np.sort(np.linalg.eigvalsh(hh)) - ref)) < 1e-12


@pytest.mark.parametrize("f", [1.0 / 8, 0.3])
def test_plaquette_flux_gauge_invariant(f):
    """The hopping phase collected around each plaquette is pi*f (electron block)
    and -pi*f (hole block), the Peierls substitution after eq. (hamil2)."""
    Lx, Ly = 6, 5
    ph = W.landau_phases(Lx, Ly, f)
    H = oracle.build_csr(Lx, Ly, 0, 0, 1.0, 0.0, np.zeros(Lx * Ly), np.zeros(Lx * Ly), None, ph)
    Hd = H.to_scipy().toarray()
    for blk, sgn in ((0, 1.0), (1, -1.0)):
        h = Hd[blk::2, blk::2]
        tt = -h if blk == 0 else h        # t_ij in the electron block, conj(t_ij) in the hole block
        for y in range(Ly - 1):
            for x in range(Lx - 1):
                s = x + Lx * y
                loop = [s, s + 1, s + 1 + Lx, s + Lx, s]
                prod = np.prod([tt[loop[i], loop[i + 1]] for i in range(4)])
                assert abs(abs(prod) - 1.0) < 1e-14
                assert abs(np.angle(prod * np.exp(-1j * sgn * np.pi * f))) < 1e-13


# -------------------------------------------------------------- kernels and weights
@pytest.mark.parametrize("N", [2, 7, 64, 1024])
def test_jackson_is_autocorrelation_of_sine_window(N):
    # Jackson's kernel is the normalised autocorrelation of the window sin(pi (k+1)/(N+1))
    av = np.sin(np.pi * (np.arange(N) + 1) / (N + 1))
    ac = np.array([np.dot(av[:N - k], av[k:]) for k in range(N)]) / np.dot(av, av)
    assert np.max(np.abs(oracle.jackson(N) - ac)) < 1e-13


def test_jackson_smoothed_delta_is_positive():
    N = 128
    g = oracle.jackson(N)
    x = np.linspace(-0.999, 0.999, 801)
    for x0 in (-0.7, 0.0, 0.31):
        mu = ed.cheb_T(np.arange(N), x0)           # moments of delta(x - x0)
        pref = np.where(np.arange(N) == 0, 1.0, 2.0)
        f = (pref * g * mu) @ ed.cheb_T(np.arange(N), x) / (np.pi * np.sqrt(1 - x * x))
        assert f.min() > -1e-12
        assert abs(np.trapezoid(f, x) - 1.0) < 2e-2


def _damped_delta_series(N, lam, x0, x):
    """sum_{n<N} (2 - delta_n0) g_n T_n(x0) T_n(x) for the Lorentz kernel,
    summed as geometric series: sinh(lam (1 - n/N)) / sinh(lam)
    = (r^n - q s^n)/(1 - q) with r = exp(-lam/N), s = exp(lam/N),
    q = exp(-2 lam), and T_n(x0) T_n(x) = [cos(n(th - th0)) + cos(n(th + th0))]/2,
    sum_{n<N} (2 - delta_n0) z^n cos(n phi) = 2 Re[(1 - (z e^{i phi})^N)/(1 - z e^{i phi})] - 1."""
    eps = lam / N
    r, s, q = np.exp(-eps), np.exp(eps), np.exp(-2.0 * lam)
    th, th0 = np.arccos(x), np.arccos(x0)

    def geo(z, phi):
        ze = z * np.exp(1j * phi)
        return 2.0 * np.real((1.0 - ze ** N) / (1.0 - ze)) - 1.0

    def series(phi):
        return (geo(r, phi) - q * geo(s, phi)) / (1.0 - q)

    return 0.5 * (series(th - th0) + series(th + th0))


def _lorentz_ldos_of_one_level(kernel_fn, N, lam, x0, x):
    """LDOS of a single level at x0 (moments mu_n = T_n(x0), a = 1, b = 0)
    through oracle.ldos with the kernel factors of kernel_fn."""
    mu = ed.cheb_T(np.arange(N), x0)[None, :]
    orig = oracle.kpm.lorentz
    try:
        oracle.kpm.lorentz = kernel_fn
        return oracle.ldos(mu, x, 1.0, 0.0, kernel="lorentz", lam=lam)[0]
    finally:
        oracle.kpm.lorentz = orig


@pytest.mark.parametrize("N,lam,x0", [(64, 5.0, 0.3), (1000, 3.0, -0.55), (4000, 4.0, 0.0)])
def test_lorentz_series_equals_geometric_closed_form(N, lam, x0):
    # The Lorentz kernel of the kernel equation after eq. (ref2) is a difference
    # of two geometric sequences in n, so the damped series of one level has a
    # closed form; pins the kernel (index and N) and the LDOS weights together.
    x = np.concatenate([np.linspace(-0.95, 0.95, 39), x0 + np.linspace(-0.01, 0.01, 21)])
    got = _lorentz_ldos_of_one_level(oracle.lorentz, N, lam, x0, x)
    ref = _damped_delta_series(N, lam, x0, x) / (np.pi * np.sqrt(1.0 - x * x))
    assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))


def test_lorentz_pin_rejects_a_misindexed_kernel():
    # a kernel shifted by one index, or normalised with N - 1 instead of N,
    # fails the closed-form check by orders of magnitude
    N, lam, x0 = 1000, 3.0, -0.55
    x = x0 + np.linspace(-0.01, 0.01, 21)
    ref = _damped_delta_series(N, lam, x0, x) / (np.pi * np.sqrt(1.0 - x * x))
    for bad in (lambda N, lam: np.sinh(lam * (1.0 - (np.arange(N) + 1.0) / N)) / np.sinh(lam),
                lambda N, lam: np.sinh(lam * (1.0 - np.arange(N) / (N - 1.0))) / np.sinh(lam)):
        got = _lorentz_ldos_of_one_level(bad, N, lam, x0, x)
        assert np.max(np.abs(got - ref)) > 1e-4 * np.max(np.abs(ref))


@pytest.mark.parametrize("N,lam", [(4000, 4.0), (40000, 8.0)])
def test_lorentz_damped_level_is_a_lorentzian(N, lam):
    # The paper's statement under the Lorentz-kernel equation: the damped series
    # of a delta function is a Lorentzian of width eps = lam/N (rescaled units).
    # At x0 = 0, to O(eps^2), the deviation is the truncation of the
    # exp(-eps n) series at n = N and the exp(-2 lam) part of the kernel, each
    # about exp(-lam) of the peak height.
    eps = lam / N
    x = np.linspace(-20 * eps, 20 * eps, 81)
    got = _lorentz_ldos_of_one_level(oracle.lorentz, N, lam, 0.0, x)
    lor = eps / np.pi / (x * x + eps * eps)
    assert np.max(np.abs(got - lor)) < 2.5 * np.exp(-lam) * np.max(lor)


@pytest.mark.parametrize("x_c", [1.0, 0.6, 0.13])
def test_sign_coefficients_by_quadrature(x_c):
    N = 41
    c = oracle.sign_coefficients(N, x_c)
    tc = np.arccos(x_c)
    for n in range(N):
        f = lambda th: np.sign(np.cos(th)) * (abs(np.cos(th)) < x_c) * np.cos(n * th)
        pts = sorted({tc, np.pi / 2, np.pi - tc})
        val, _ = integrate.quad(f, 0, np.pi, points=pts, limit=400, epsabs=1e-13)
        ref = (1 if n == 0 else 2) / np.pi * val
        assert abs(c[n] - ref) < 1e-11, n


@pytest.mark.parametrize("a,b,E_c", [(3.0, 0.0, 0.0), (3.0, 0.4, 0.0), (2.5, -0.3, 1.1), (4.0, 0.2, 9.0)])
def test_general_sign_weight_by_quadrature(a, b, E_c):
    """sign(E) on |E| < E_c with E = a x + b, integrated against T_n numerically."""
    N = 33
    c = oracle.sign_weight_coefficients(N, a, b, E_c)
    for n in range(N):
        def f(th):
            E = a * np.cos(th) + b
            inside = (abs(E) < E_c) if E_c > 0 else True
            return np.sign(E) * inside * np.cos(n * th)
        pts = [np.arccos(np.clip(v, -1, 1)) for v in (-b / a, (E_c - b) / a, (-E_c - b) / a)]
        val, _ = integrate.quad(f, 0, np.pi, points=sorted(set(pts)), limit=400, epsabs=1e-13)
        assert abs(c[n] - (1 if n == 0 else 2) / np.pi * val) < 1e-11, n
    if b == 0.0:
        x_c = min(E_c / a, 1.0) if E_c > 0 else 1.0
        assert np.max(np.abs(c - oracle.sign_coefficients(N, x_c))) < 1e-14


def test_sign_series_converges_to_sign():
    c = oracle.sign_coefficients(4001)
    x = np.array([-0.9, -0.5, -0.2, 0.3, 0.8])
    val = c @ ed.cheb_T(np.arange(4001), x)
    assert np.max(np.abs(val - np.sign(x))) < 2e-2


# ------------------------------------------------- P8 / P9: gap equation vs ED
def test_gap_map_equals_ed_with_same_polynomial_filter():
    w = W.config0()
    _, _, a, b = oracle.workload_bounds(w)
    _, mu_he = oracle.workload_moments(w, a, b)
    new = oracle.gap_map(mu_he, w.U).real
    Et, V = ed.eig(w, a, b)
    p = np.polynomial.chebyshev.chebval(Et, oracle.gap_weights(w.N))
    u, v = V[:w.L2], V[w.L2:]
    ref = 0.5 * w.U * np.sum(u * np.conj(v) * p[None, :], axis=1)
    assert np.max(np.abs(new - ref.real)) < 1e-13
    assert np.max(np.abs(ref.imag)) < 1e-13


def test_gap_map_complex_delta_equals_ed():
    """With a complex gap the conjugation matters: Delta_i = (U/2) sum_k u_k(i) conj(v_k(i)) p(E_k)."""
    w = _small(seed=17, complex_=True, bond=True, flux=0.2)
    _, _, a, b = oracle.workload_bounds(w)
    N = 120
    _, mu_he = oracle.workload_moments(w, a, b, N=N)
    new = oracle.gap_map(mu_he, w.U)
    Et, V = ed.eig(w, a, b)
    p = np.polynomial.chebyshev.chebval(Et, oracle.gap_weights(N))
    ref = 0.5 * w.U * np.sum(V[:w.L2] * np.conj(V[w.L2:]) * p[None, :], axis=1)
    assert np.max(np.abs(ref.imag)) > 1e-3          # genuinely complex
    assert np.max(np.abs(new - ref)) < 1e-13


def test_gap_map_approaches_exact_ed_with_growing_N():
    """Physics check, tolerance-bounded: the damped series converges to the
    exact T = 0 sign weight as N grows."""
    w = W.config0()
    _, _, a, b = oracle.workload_bounds(w)
    Et, V = ed.eig(w, a, b)
    exact = 0.5 * w.U * np.sum(V[:w.L2] * V[w.L2:] * np.sign(Et)[None, :], axis=1)
    errs = []
    for N in (128, 512, 2048):
        _, mu_he = oracle.workload_moments(w, a, b, N=N)
        errs.append(np.max(np.abs(oracle.gap_map(mu_he, w.U).real - exact)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 5e-3


def test_atomic_limit_gap_is_bcs():
    # t = 0: one site obeys Delta = (U/2) Delta / sqrt(xi^2 + Delta^2)
    xi, U = 0.3, 2.0
    dstar = np.sqrt((U / 2) ** 2 - xi ** 2)
    w = W.Workload("bcs", 1, 1, W.OPEN, W.OPEN, 0.0, -xi, U, np.zeros(1), np.array([dstar]),
                   None, None, 4096, np.array([0], np.int32), 1)
    a = 2.0
    _, mu_he = oracle.workload_moments(w, a, 0.0)
    new = oracle.gap_map(mu_he, U).real
    assert abs(new[0] - dstar) < 1e-3


# ------------------------------------------------------------------------ LDOS
def test_ldos_equals_kernel_broadened_ed():
    w = _small(seed=21)
    _, _, a, b = oracle.workload_bounds(w)
    N = 200
    mu_ee, _ = oracle.workload_moments(w, a, b, N=N)
    E = np.linspace(-2.5, 2.5, 37)
    got = oracle.ldos(mu_ee, E, a, b)
    Et, V = ed.eig(w, a, b)
    g = oracle.jackson(N)
    x = (E - b) / a
    # sum_k |u_k(i)|^2 K_N(x, E_k) with the Jackson-damped delta kernel, per unit energy
    Tx = ed.cheb_T(np.arange(N), x)                                  # [N, m]
    Tk = ed.cheb_T(np.arange(N), Et)                                 # [N, D]
    pref = np.where(np.arange(N) == 0, 1.0, 2.0) * g
    K = (Tk.T * pref) @ Tx / (np.pi * np.sqrt(1 - x * x))[None, :] / a    # [D, m]
    ref = (np.abs(V[:w.L2]) ** 2) @ K
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    # normalisation: the LDOS integrates to mu_0 = 1 over the band (up to damping tails)
    Ef = np.linspace(-a * 0.999, a * 0.999, 20001)
    tot = np.trapezoid(oracle.ldos(mu_ee[:3], Ef, a, b), Ef, axis=1)
    assert np.max(np.abs(tot - 1.0)) < 2e-2


def _panel_integral(f, lo, hi, h):
    """int_lo^hi f(E) dE with 8-point Gauss-Legendre panels of width <= h;
    f maps an array of energies to [len(E), rows]."""
    xg, wg = np.polynomial.legendre.leggauss(8)
    edges = np.linspace(lo, hi, int(np.ceil((hi - lo) / h)) + 1)
    mid, half = 0.5 * (edges[1:] + edges[:-1]), 0.5 * (edges[1:] - edges[:-1])
    pts = (mid[:, None] + half[:, None] * xg[None, :]).ravel()
    return (half[:, None] * wg[None, :]).ravel() @ f(pts)


def _ldos_level_weight_error(ldos_fn):
    """Largest error of the spectral weight the LDOS puts around each isolated
    level: int over [midpoint to the level below, midpoint to the level above]
    of N_up(E, i) dE must equal |u_k(i)|^2 (eq. (imag1): the spectral function
    is sum_k |u_k(i)|^2 delta(E - E_k)), up to the Jackson kernel's tails,
    which at a distance of 30 kernel widths are far below 1e-5."""
    w = W.small_random(3, 2, N=64, seed=5)
    _, _, a, b = oracle.workload_bounds(w)
    Et, V = ed.eig(w, a, b)
    E = Et * a + b
    N = 4096
    mu_ee, _ = oracle.workload_moments(w, a, b, N=N)
    sig = a * np.pi / N                       # Jackson resolution in energy
    errs = []
    for k in range(len(E)):
        if (k > 0 and E[k] - E[k - 1] < 60 * sig) or (k + 1 < len(E) and E[k + 1] - E[k] < 60 * sig):
            continue
        lo = 0.5 * (E[k - 1] + E[k]) if k > 0 else b - 0.9999 * a
        hi = 0.5 * (E[k + 1] + E[k]) if k + 1 < len(E) else b + 0.9999 * a
        got = _panel_integral(lambda e: ldos_fn(mu_ee, e, a, b).T, lo, hi, sig / 2)
        errs.append(np.max(np.abs(got - np.abs(V[:w.L2, k]) ** 2)))
    assert len(errs) >= 8
    return max(errs)


def test_ldos_puts_each_levels_weight_around_it():
    # eq. (ldos) with eq. (imag2): the n >= 1 terms carry a factor 2 against
    # n = 0 (a_n = mu_n / (1 + delta_n0)); the integrated weight of one level
    # depends on every term of the series
    assert _ldos_level_weight_error(oracle.ldos) < 1e-5


def test_ldos_weight_pin_rejects_a_dropped_factor_two():
    # a copy of the oracle's LDOS with the factor 2 on n >= 1 replaced by 1
    def dropped(mu_ee, energies, a, b):
        N = mu_ee.shape[-1]
        x = (np.asarray(energies) - b) / a
        T = ed.cheb_T(np.arange(N), x).T
        return mu_ee @ (T * oracle.jackson(N)[None, :] / (np.pi * a * np.sqrt(1 - x * x))[:, None]).T
    assert _ldos_level_weight_error(dropped) > 1e-2


# ---------------------------------------------- P10 / P11 / P12: gradients
def _dk_gradient(w, a, b, sites, w_ee, w_he):
    """Daleckii-Krein derivative of L = sum_s <s,e|p_ee(Ht)|s,e> + <s,h|p_he(Ht)|s,e>."""
    Et, V = ed.eig(w, a, b)
    N = w_ee.shape[-1]
    L2 = w.L2
    D1 = ed.cheb_divided_difference(np.arange(N), Et[:, None], Et[None, :])   # [N, D, D]
    ge = np.zeros(L2)
    gd = np.zeros(L2)
    # B = V^T M V with M = sum_s |s,e><bra_s|, weighted per n
    P1 = np.zeros((len(Et), len(Et)))
    Bsum = np.zeros((len(Et), len(Et)))
    for q, s in enumerate(sites):
        ket = V[s, :]
        for wn, brarow in ((w_ee[q], V[s, :]), (w_he[q], V[L2 + s, :])):
            pk = np.tensordot(wn, D1, axes=(0, 0))                     # [D, D] p^[1]
            # d<bra|p(H)|ket> = sum_kl bra_k A_kl ket_l p1_kl with A = V^T dH V
            Bsum += np.outer(brarow, ket) * pk
    Ve, Vh = V[:L2], V[L2:]
    for j in range(L2):
        Ae = (np.outer(Ve[j], Ve[j]) - np.outer(Vh[j], Vh[j])) / a
        Ad = (np.outer(Ve[j], Vh[j]) + np.outer(Vh[j], Ve[j])) / a
        ge[j] = np.sum(Ae * Bsum)
        gd[j] = np.sum(Ad * Bsum)
    return ge, gd


def _loss_weights(w, a, N, sites):
    rng = np.random.default_rng(9)
    return rng.normal(size=(len(sites), N)), rng.normal(size=(len(sites), N))


def test_backward_equals_daleckii_krein():
    w = W.small_random(6, 5, N=40, seed=8, n_sites=7)
    _, _, a, b = oracle.workload_bounds(w)
    N = 40
    w_ee, w_he = _loss_weights(w, a, N, w.start_sites)
    H = oracle.workload_csr(w, a, b)
    ge, gd = oracle.moments_backward(H, w.start_sites, N, w_ee, w_he)
    re, rd = _dk_gradient(w, a, b, w.start_sites, w_ee, w_he)
    scale = max(np.max(np.abs(re)), np.max(np.abs(rd)))
    assert np.max(np.abs(ge - re)) < 1e-12 * scale
    assert np.max(np.abs(gd - rd)) < 1e-12 * scale


def test_backward_equals_richardson_finite_differences():
    w = W.small_random(5, 4, N=30, seed=12, n_sites=5)
    _, _, a, b = oracle.workload_bounds(w)
    N = 30
    w_ee, w_he = _loss_weights(w, a, N, w.start_sites)
    H = oracle.workload_csr(w, a, b)
    ge, gd = oracle.moments_backward(H, w.start_sites, N, w_ee, w_he)

    def loss(eps, delta):
        Hq = oracle.build_csr(w.Lx, w.Ly, w.bc_x, w.bc_y, w.t, w.mu_c, eps, delta, None, None, a, b)
        me, mh = oracle.moments(Hq, w.start_sites, N)
        return np.sum(w_ee * me) + np.sum(w_he * mh)

    def fd(j, which, h):
        e, d = w.eps.copy(), np.array(w.delta, dtype=float)
        arr = e if which == 0 else d
        arr[j] += h
        lp = loss(e, d)
        arr[j] -= 2 * h
        lm = loss(e, d)
        return (lp - lm) / (2 * h)

    for j in range(w.L2):
        for which, g in ((0, ge), (1, gd)):
            h = 1e-3
            rich = (4 * fd(j, which, h / 2) - fd(j, which, h)) / 3
            assert abs(g[j] - rich) < 1e-8 * max(1.0, abs(rich)), (j, which)


def test_gap_jacobian_is_symmetric():
    """J_F[i,j] = dF_i/dDelta_j of the gap map is symmetric for a real operator
    and uniform U, so one reverse pass serves as a Jacobian-vector product."""
    w = W.small_random(4, 4, N=48, seed=2)
    _, _, a, b = oracle.workload_bounds(w)
    N = 48
    H = oracle.workload_csr(w, a, b)
    wg = 0.5 * w.U * oracle.gap_weights(N)
    J = np.zeros((w.L2, w.L2))
    for i in range(w.L2):
        dmu_he = np.zeros((w.L2, N))
        dmu_he[i] = wg
        _, gd = oracle.moments_backward(H, w.start_sites, N, np.zeros((w.L2, N)), dmu_he)
        J[i] = gd
    assert np.max(np.abs(J - J.T)) < 1e-13 * np.max(np.abs(J))


# ---------------------------------------------------------------------- SCF
def test_scf_matches_ed_self_consistency_with_same_filter():
    """The oracle's plain-mixing fixed point is a fixed point of the ED gap map
    with the same polynomial filter."""
    w = W.config0()
    delta, it, r, (a, b) = oracle.scf_plain(w, tol=1e-10, max_iter=300)
    assert r < 1e-10
    Et, V = ed.eig(w, a, b, delta)
    p = np.polynomial.chebyshev.chebval(Et, oracle.gap_weights(w.N))
    ref = 0.5 * w.U * np.sum(V[:w.L2] * V[w.L2:] * p[None, :], axis=1)
    assert np.max(np.abs(ref - delta)) < 1e-9
    # the impurity suppresses the gap locally
    assert delta[W.site(16, 8, 8)] < delta[W.site(16, 2, 2)]


# ----------------------------------------------- moment doubling identities
def _vectors(H, s, K):
    """a_0..a_K of one start vector through the oracle's explicit matrix."""
    import scipy.sparse as sp
    A = H.to_scipy()
    a = [np.zeros(H.D, dtype=np.complex128)]
    a[0][2 * s] = 1.0
    a.append(A @ a[0])
    for n in range(2, K + 1):
        a.append(2 * (A @ a[-1]) - a[-2])
    return a


@pytest.mark.parametrize("case", [dict(), dict(complex_=True, bond=True, flux=0.2)])
def test_moment_doubling_identities(case):
    """With b = 0 and C(u,v) = (-v*, u*) anticommuting with Ht:
    mu_ee[2n] = 2<a_n|a_n> - mu_0, mu_ee[2n-1] = 2<a_n|a_{n-1}> - mu_ee[1],
    mu_he[2n-1] = 2(-1)^n B(a_n, a_{n-1}) - mu_he[1], mu_he[2n] = 0,
    with the bilinear form B(a, b) = sum_i u_a(i) v_b(i) - v_a(i) u_b(i)."""
    w = _small(**case)
    _, _, a, b = oracle.workload_bounds(w)
    assert b == 0.0
    K = 30
    H = oracle.workload_csr(w, a, b)
    for s in (0, 7, w.L2 - 1):
        mu_ee, mu_he = oracle.moments(H, [s], 2 * K + 1, force_complex=True)
        vec = _vectors(H, s, K)
        for n in range(1, K + 1):
            an, am = vec[n], vec[n - 1]
            assert abs(2 * np.vdot(an, an).real - mu_ee[0, 0] - mu_ee[0, 2 * n]) < 1e-13
            assert abs(2 * np.vdot(an, am).real - mu_ee[0, 1] - mu_ee[0, 2 * n - 1]) < 1e-13
            u_n, v_n, u_m, v_m = an[0::2], an[1::2], am[0::2], am[1::2]
            B = np.sum(u_n * v_m - v_n * u_m)
            assert abs(2 * (-1) ** n * B - mu_he[0, 1] - mu_he[0, 2 * n - 1]) < 1e-13
            assert abs(mu_he[0, 2 * n]) < 1e-13


# ------------------------------------------- finite temperature and density
def test_thermal_coefficients_reduce_to_closed_forms_at_zero_temperature():
    """T = 0: the quadrature gives the closed-form sign coefficients (pinned
    above) and, for the density, those of theta(-E) written out here."""
    N, a, b = 64, 5.3, 0.4
    for E_c in (0.0, 2.1):
        q = oracle.thermal_coefficients(N, a, b, 0.0, E_c, "gap")
        assert np.max(np.abs(q - oracle.sign_weight_coefficients(N, a, b, E_c))) < 1e-10
    q = oracle.thermal_coefficients(N, a, b, 0.0, quantity="density")
    t0 = np.arccos(-b / a)
    n = np.arange(1, N)
    closed = np.concatenate([[(np.pi - t0) / np.pi], -2.0 * np.sin(n * t0) / (np.pi * n)])
    assert np.max(np.abs(q - closed)) < 1e-10
    # and a small temperature stays within O(T/a) of the step
    qs = oracle.thermal_coefficients(N, a, b, 1e-4, quantity="density")
    assert np.max(np.abs(qs - closed)) < 1e-4


@pytest.mark.parametrize("quantity,T", [("gap", 0.3), ("density", 0.3)])
def test_thermal_series_reconstructs_the_weight(quantity, T):
    """Smooth weights: sum_n c_n T_n(x) converges to the weight itself, so the
    c_n are its Chebyshev coefficients."""
    a, b, N = 4.7, -0.3, 600
    c = oracle.thermal_coefficients(N, a, b, T, 0.0, quantity)
    x = np.linspace(-0.95, 0.95, 41)
    E = a * x + b
    w = np.tanh(E / (2 * T)) if quantity == "gap" else 1.0 / (np.exp(E / T) + 1.0)
    series = np.polynomial.chebyshev.chebval(x, c)
    assert np.max(np.abs(series - w)) < 1e-6


def test_thermal_gap_coefficients_with_cutoff_equal_discrete_transform():
    """With a cutoff the weight jumps at |E| = E_c; compare with the discrete
    Chebyshev transform on M Chebyshev-Gauss nodes, whose error from the jumps
    is O(1/M)."""
    a, b, T, E_c, N, M = 4.7, -0.3, 0.5, 2.5, 200, 400000
    c = oracle.thermal_coefficients(N, a, b, T, E_c, "gap")
    t = np.pi * (np.arange(M) + 0.5) / M
    E = a * np.cos(t) + b
    w = np.tanh(E / (2 * T)) * (np.abs(E) < E_c)
    n = np.arange(N)
    d = np.where(n == 0, 1.0, 2.0) / M * (np.cos(np.outer(n, t)) @ w)
    assert np.max(np.abs(c - d)) < 2e-5


def test_finite_temperature_gap_and_density_approach_exact_ed():
    """Physics checks against exact diagonalisation at T = 0.25: the error is
    the Jackson broadening (width ~ pi a/N, much smaller than T), so it falls
    as 1/N^2 -- 16x from N = 256 to 1024 (measured 2.1e-3 -> 1.4e-4):
    Delta_i = (U/2) sum_k u_k(i) conj(v_k(i)) tanh(E_k/2T) and
    n_i = 2 sum_k |u_k(i)|^2 f(E_k)."""
    w = _small(Lx=4, Ly=4, seed=31)
    _, _, a, b = oracle.workload_bounds(w)
    T = 0.25
    Et, V = ed.eig(w, a, b)
    E = a * Et + b
    L2 = w.L2
    exact_gap = 0.5 * w.U * np.sum(V[:L2] * np.conj(V[L2:]) * np.tanh(E / (2 * T))[None, :], axis=1).real
    exact_n = 2.0 * np.sum(np.abs(V[:L2]) ** 2 / (np.exp(E / T) + 1.0)[None, :], axis=1)
    errs = []
    for N in (256, 1024):
        mu_ee, mu_he = oracle.workload_moments(w, a, b, N=N)
        g = oracle.gap_map_thermal(mu_he, w.U, a, b, T).real
        n = oracle.density(mu_ee, a, b, T)
        errs.append((np.max(np.abs(g - exact_gap)), np.max(np.abs(n - exact_n))))
    assert errs[0][0] > 12 * errs[1][0] and errs[0][1] > 12 * errs[1][1]
    assert errs[1][0] < 3e-4 and errs[1][1] < 3e-4


def test_density_of_a_free_lattice_counts_filled_states():
    """Delta = 0, eps = 0: at T -> 0 the total electron number is twice the
    number of tight-binding levels below mu (open square lattice, levels
    -2t(cos(k_x) + cos(k_y)) with k = pi m/(L+1)); moments by the oracle,
    N large."""
    L, mu = 6, -0.3
    w = W.Workload("free", L, L, W.OPEN, W.OPEN, 1.0, mu, 0.0, np.zeros(L * L), np.zeros(L * L),
                   None, None, 2048, np.arange(L * L, dtype=np.int32), L * L)
    a, b = 4.4, 0.0
    mu_ee, _ = oracle.workload_moments(w, a, b)
    n = oracle.density(mu_ee, a, b, T=0.02)
    k = np.pi * np.arange(1, L + 1) / (L + 1)
    levels = (-2 * (np.cos(k)[:, None] + np.cos(k)[None, :])).ravel() - mu
    assert np.min(np.abs(levels)) > 0.1                     # no level near E = 0
    assert abs(np.sum(n) - 2 * np.sum(levels < 0)) < 1e-3


# ------------------------------------------- neighbour moments, bonds, current
@pytest.mark.parametrize("case", [dict(), dict(bc_x=W.PERIODIC, bc_y=W.PERIODIC),
                                  dict(complex_=True, bond=True, flux=0.2, bc_x=W.PERIODIC)])
def test_neighbour_moments_equal_exact_diagonalisation(case):
    """<j,alpha|T_n(Ht)|i,e> = sum_k V[j alpha, k] conj(V[i e, k]) T_n(E_k)."""
    w = _small(Lx=5, Ly=4, seed=41, **case)
    _, _, a, b = oracle.workload_bounds(w)
    H = oracle.workload_csr(w, a, b)
    N = 24
    sites = np.array([0, 7, w.L2 - 1])
    ee, he = oracle.neighbour_moments(H, w.Lx, w.Ly, w.bc_x, w.bc_y, sites, N)
    Et, V = ed.eig(w, a, b)
    T = ed.cheb_T(np.arange(N), Et)            # [N, D]
    L2 = w.L2
    for k, s in enumerate(sites):
        for d in range(4):
            j = oracle.neighbour_site(w.Lx, w.Ly, w.bc_x, w.bc_y, int(s), d)
            if j < 0:
                assert np.all(ee[k, d] == 0) and np.all(he[k, d] == 0)
                continue
            ref_e = (V[j] * np.conj(V[s])) @ T.T
            ref_h = (V[L2 + j] * np.conj(V[s])) @ T.T
            assert np.max(np.abs(ee[k, d] - ref_e)) < 1e-12
            assert np.max(np.abs(he[k, d] - ref_h)) < 1e-12


def test_bond_gap_map_equals_bloch_closed_form():
    """Periodic lattice with uniform d-wave bonds Delta_x = D0, Delta_y = -D0.
    Per k the 2x2 block [[xi_k, D(k)], [D(k), -xi_k]], D(k) = 2 D0 (cos kx -
    cos ky), and an odd polynomial filter p acts as p(E_k) H(k)/E_k, so
    <j,h|p(Ht)|i,e> = (1/L^2) sum_k e^{ik(r_i - r_j)} D(k) p(E_k/a)/E_k and the
    bond map is (U/4)(conj S_+x + conj S_-x) -- exact for any N."""
    L, t, mu, D0, U, N = 8, 1.0, -0.3, 0.15, 1.7, 64
    L2 = L * L
    db = np.zeros((2, L2), dtype=np.complex128)
    db[0], db[1] = D0, -D0
    w = W.Workload("dwave", L, L, W.PERIODIC, W.PERIODIC, t, mu, U, np.zeros(L2), np.zeros(L2), db,
                   None, N, np.arange(L2, dtype=np.int32), L2, scalar="complex", pairing="bond")
    a = 6.3
    H = oracle.workload_csr(w, a, 0.0)
    ee, he = oracle.neighbour_moments(H, L, L, 1, 1, np.arange(L2), N)
    wts = oracle.gap_weights(N)
    out = oracle.bond_gap_map(he, U, L, L, 1, 1, wts)
    k = 2 * np.pi * np.arange(L) / L
    kx, ky = np.meshgrid(k, k, indexing="ij")
    xi = -2 * t * (np.cos(kx) + np.cos(ky)) - mu
    Dk = 2 * D0 * (np.cos(kx) - np.cos(ky))
    E = np.sqrt(xi ** 2 + Dk ** 2)
    p = np.polynomial.chebyshev.chebval(E / a, wts)
    Sx = np.mean(np.exp(-1j * kx) * Dk * p / E)      # <i+x,h|p|i,e>
    Sxm = np.mean(np.exp(1j * kx) * Dk * p / E)      # <i-x,h|p|i,e>
    Sy = np.mean(np.exp(-1j * ky) * Dk * p / E)
    Sym = np.mean(np.exp(1j * ky) * Dk * p / E)
    assert np.max(np.abs(out[0] - 0.25 * U * (np.conj(Sx) + np.conj(Sxm)))) < 1e-12
    assert np.max(np.abs(out[1] - 0.25 * U * (np.conj(Sy) + np.conj(Sym)))) < 1e-12
    assert np.max(np.abs(out[0] + out[1])) < 1e-12          # d-wave: Delta_y = -Delta_x


def test_bond_current_vanishes_without_flux_and_is_conserved_with_it():
    """Real operator: <c_i^+ c_j> is real, no current.  Delta = 0 with flux:
    p(Ht) commutes with Ht, so the currents out of every site add to zero."""
    w = _small(Lx=6, Ly=5, seed=43)
    _, _, a, b = oracle.workload_bounds(w)
    N = 200
    H = oracle.workload_csr(w, a, b)
    ee, _ = oracle.neighbour_moments(H, w.Lx, w.Ly, w.bc_x, w.bc_y, np.arange(w.L2), N)
    wf = oracle.jackson(N) * oracle.thermal_coefficients(N, a, b, 0.05, quantity="density")
    J = oracle.bond_current(ee, w.t, None, w.Lx, w.Ly, w.bc_x, w.bc_y, wf)
    assert np.max(np.abs(J)) < 1e-13
    wn = _small(Lx=6, Ly=5, seed=44, complex_=True, flux=0.15)
    wn = wn.with_(delta=np.zeros(wn.L2, dtype=np.complex128))
    _, _, a, b = oracle.workload_bounds(wn)
    H = oracle.workload_csr(wn, a, b)
    ee, _ = oracle.neighbour_moments(H, wn.Lx, wn.Ly, wn.bc_x, wn.bc_y, np.arange(wn.L2), N)
    wf = oracle.jackson(N) * oracle.thermal_coefficients(N, a, b, 0.05, quantity="density")
    J = oracle.bond_current(ee, wn.t, wn.peierls, wn.Lx, wn.Ly, wn.bc_x, wn.bc_y, wf)
    assert np.max(np.abs(J)) > 1e-3
    div = J[0] + J[1]
    for s in range(wn.L2):
        for axis, back in ((0, 1), (1, 3)):
            j = oracle.neighbour_site(wn.Lx, wn.Ly, wn.bc_x, wn.bc_y, s, back)
            if j >= 0:
                div[s] -= J[axis, j]
    assert np.max(np.abs(div)) < 1e-12


def test_ring_current_is_the_flux_derivative_of_the_grand_potential():
    """A periodic 9x3 lattice at T = 0.1 with phase theta on every x bond: by
    Hellmann-Feynman the x-bond currents add up to dOmega/dtheta, with the
    grand potential Omega = -2T sum_k ln(1 + exp(-(eps_k - mu)/T)) of the
    levels eps = -2t cos(kx + theta) - 2t cos(ky) (a particle's velocity is
    d eps/d theta).  The Jackson broadening makes the error fall as 1/N^2
    (measured 6.7e-3, 1.7e-3, 4.3e-4 at N = 800, 1600, 3200)."""
    Lx, Ly, t, mu, T, th = 9, 3, 1.0, -0.35, 0.1, 0.21
    L2 = Lx * Ly
    ph = np.zeros((2, L2))
    ph[0] = th

    def omega(theta):
        kx = 2 * np.pi * np.arange(Lx) / Lx
        ky = 2 * np.pi * np.arange(Ly) / Ly
        e = (-2 * t * np.cos(kx[:, None] + theta) - 2 * t * np.cos(ky[None, :])).ravel() - mu
        return -2 * T * np.sum(np.log1p(np.exp(-e / T)))
    h = 1e-5
    dO = (omega(th + h) - omega(th - h)) / (2 * h)
    errs = []
    for N in (800, 1600):
        w = W.Workload("ring", Lx, Ly, W.PERIODIC, W.PERIODIC, t, mu, 0.0, np.zeros(L2),
                       np.zeros(L2, np.complex128), None, ph, N, np.arange(L2, dtype=np.int32), L2,
                       scalar="complex")
        a = 4.6
        H = oracle.workload_csr(w, a, 0.0)
        ee, _ = oracle.neighbour_moments(H, Lx, Ly, 1, 1, np.arange(L2), N)
        wf = oracle.jackson(N) * oracle.thermal_coefficients(N, a, 0.0, T, quantity="density")
        J = oracle.bond_current(ee, t, ph, Lx, Ly, 1, 1, wf)
        assert np.max(np.abs(J[1])) < 1e-12                       # no flux on y bonds
        assert np.max(np.abs(J[0] - J[0].mean())) < 1e-10          # uniform
        errs.append(abs(J[0].sum() - dO))
    assert errs[0] > 3.5 * errs[1]
    assert errs[1] < 0.04 * abs(dO)
