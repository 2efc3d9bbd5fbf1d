"""Kernel factors, energy weights and observables in NumPy FP64 (test oracle).

Conventions: moments mu_n are <bra|T_n(Ht)|s,e> for n = 0..N-1 (no
1/(1+delta_{0n}) factor), Ht = (H - b)/a, energies are in units of t.
"""
from __future__ import annotations

import numpy as np


def jackson(N: int) -> np.ndarray:
    """Jackson kernel factors g_n, n = 0..N-1.

    The paper damps the truncated series with a kernel (paragraph before the
    Lorentz-kernel equation); the Jackson form is the one of its KPM reference
    (weisse2006): g_n = [(N-n+1) cos(pi n/(N+1)) + sin(pi n/(N+1)) cot(pi/(N+1))]/(N+1).
    """
    n = np.arange(N, dtype=np.float64)
    q = np.pi / (N + 1)
    return ((N - n + 1) * np.cos(q * n) + np.sin(q * n) / np.tan(q)) / (N + 1)


def lorentz(N: int, lam: float) -> np.ndarray:
    """Lorentz kernel factors sinh[lam (1 - n/N)] / sinh(lam) (the kernel
    equation following eq. (ref2)); the broadening is eps = lam/N in rescaled
    energy units."""
    n = np.arange(N, dtype=np.float64)
    return np.sinh(lam * (1.0 - n / N)) / np.sinh(lam)


def chebyshev_T(n, x):
    """T_n(x) = cos(n arccos x) on [-1, 1] (definition under the expansion of
    f(x) in Chebyshev polynomials)."""
    return np.cos(np.multiply.outer(np.asarray(n, dtype=np.float64), np.arccos(x)))


def sign_coefficients(N: int, x_c: float = 1.0) -> np.ndarray:
    """Chebyshev coefficients c_n of w(x) = 1 - 2 f = sign(x) on |x| < x_c,
    w = 0 outside, so that w(x) = sum_n c_n T_n(x) (T = 0 limit of the weight
    (1 - 2 f(E)) in eq. (op1); x_c = E_c/a is the rescaled cutoff).

    With x = cos(theta):  c_n = (2/pi) int_0^pi w(cos theta) cos(n theta) dtheta
    = 4 [sin(n pi/2) - sin(n arccos x_c)] / (n pi) for odd n, 0 for even n.
    Reading: E_c is not fixed by the workloads, so the default is no cutoff.
    """
    c = np.zeros(N)
    n = np.arange(1, N, dtype=np.float64)
    tc = np.arccos(min(max(x_c, -1.0), 1.0))
    odd = (np.arange(1, N) % 2) == 1
    c[1:][odd] = 4.0 * (np.sin(n[odd] * np.pi / 2) - np.sin(n[odd] * tc)) / (n[odd] * np.pi)
    return c


def sign_weight_coefficients(N: int, a: float = 1.0, b: float = 0.0, E_c: float = 0.0) -> np.ndarray:
    """Chebyshev coefficients of w(x) = sign(E) on |E| < E_c (E_c <= 0: no
    cutoff), E = a x + b, the T = 0 weight (1 - 2f(E)) of eq. (op1) for any
    rescaling.  With x = cos(theta) the weight is piecewise constant in theta:
    +1 between acos(x_hi) and acos(x_0), -1 between acos(x_0) and acos(x_lo),
    x_0 = -b/a, x_hi = (E_c - b)/a, x_lo = (-E_c - b)/a clipped to [-1, 1];
    each piece integrates cos(n theta) exactly.
    """
    x0 = -b / a
    if E_c > 0:
        xhi, xlo = min((E_c - b) / a, 1.0), max((-E_c - b) / a, -1.0)
    else:
        xhi, xlo = 1.0, -1.0
    pieces = [(np.arccos(xhi), np.arccos(x0), 1.0), (np.arccos(x0), np.arccos(xlo), -1.0)]
    n = np.arange(N, dtype=np.float64)
    c = np.zeros(N)
    for lo, hi, val in pieces:
        c[0] += val * (hi - lo) / np.pi
        c[1:] += val * 2.0 / np.pi * (np.sin(n[1:] * hi) - np.sin(n[1:] * lo)) / n[1:]
    return c


def gap_weights(N: int, kernel: str = "jackson", lam: float = 0.0, x_c: float = 1.0,
                a: float = None, b: float = 0.0, E_c: float = 0.0):
    """g_n c_n of the gap equation.  With a given, the general weight
    sign(E) on |E| < E_c for the rescaling (a, b); else the b = 0 closed form
    with rescaled cutoff x_c."""
    g = jackson(N) if kernel == "jackson" else lorentz(N, lam)
    if a is not None:
        return g * sign_weight_coefficients(N, a, b, E_c)
    return g * sign_coefficients(N, x_c)


def gap_map(mu_he, U, N=None, kernel="jackson", lam=0.0, x_c=1.0, a=None, b=0.0, E_c=0.0):
    """On-site order parameter from eq. (op1) at T = 0.

    Reading of the printed prefactor (garbled in the source): with the
    Bogoliubov eigenvectors (u_k(i), v_k(i)) = (<i,e|k>, <i,h|k>),
    Delta_i = U <c_{i,up} c_{i,down}> = (U/2) sum_k u_k(i) conj(v_k(i)) tanh(E_k/2T),
    which at T = 0 is (U/2) conj(<i,h| sign(H) |i,e>).  The sign function is
    replaced by its damped Chebyshev series sum_n g_n c_n T_n(Ht), so
        Delta_i^new = (U/2) conj( sum_n g_n c_n mu^he_n(i) ).
    U may be a scalar or a per-row array.
    """
    mu_he = np.asarray(mu_he)
    N = mu_he.shape[-1] if N is None else N
    w = gap_weights(N, kernel, lam, x_c, a, b, E_c)
    s = mu_he @ w
    return 0.5 * np.asarray(U) * np.conj(s)


def ldos_weights(N: int, energies, a: float, b: float, kernel: str = "jackson", lam: float = 0.0):
    """W[m, n] with N_up(E_m, i) = sum_n W[m, n] mu^ee_n(i), from eq. (ldos) and
    eq. (imag2):  -(1/pi) Im G^11_ii = [g_0 mu_0 + 2 sum_{n>=1} g_n mu_n T_n(Et)]
    / (pi sqrt(1 - Et^2)) per unit of Et, divided by a for energy units,
    with Et = (E - b)/a."""
    g = jackson(N) if kernel == "jackson" else lorentz(N, lam)
    et = (np.asarray(energies, dtype=np.float64) - b) / a
    T = chebyshev_T(np.arange(N), et).T           # [m, n]
    pref = np.where(np.arange(N) == 0, 1.0, 2.0) * g
    return T * pref[None, :] / (np.pi * a * np.sqrt(1.0 - et * et))[:, None]


def ldos(mu_ee, energies, a, b, kernel="jackson", lam=0.0):
    """Local density of states per spin, N_up(E_m, i) for every row i of mu_ee.
    Returns [rows, n_E]."""
    mu_ee = np.asarray(mu_ee, dtype=np.float64)
    W = ldos_weights(mu_ee.shape[-1], energies, a, b, kernel, lam)
    return mu_ee @ W.T


def _theta(x):
    return float(np.arccos(min(max(x, -1.0), 1.0)))


def thermal_coefficients(N: int, a: float, b: float, T: float, E_c: float = 0.0,
                         quantity: str = "gap") -> np.ndarray:
    """Chebyshev coefficients c_n of the energy weights at temperature T, so
    that w(a x + b) = sum_n c_n T_n(x) on [-1, 1]:
      quantity "gap":     w(E) = 1 - 2 f(E) = tanh(E / 2T) on |E| < E_c (E_c <= 0:
                          no cutoff), 0 outside -- the weight of eq. (op1);
      quantity "density": w(E) = f(E) = 1 / (exp(E/T) + 1) -- the weight of the
                          electron-density equation.
    c_n = ((2 - delta_n0)/pi) int_0^pi w(a cos t + b) cos(n t) dt, each
    integral by adaptive quadrature for the cosine weight (scipy QAWO),
    split where w changes fastest (E = 0) and at the cutoff.  T = 0 gives
    the step functions sign(E) and theta(-E).
    """
    from scipy import integrate
    lo, hi = 0.0, np.pi
    if quantity == "gap":
        if E_c > 0:
            lo, hi = _theta((E_c - b) / a), _theta((-E_c - b) / a)
        if T > 0:
            def w(t):
                return np.tanh((a * np.cos(t) + b) / (2.0 * T))
        else:
            def w(t):
                return np.sign(a * np.cos(t) + b)
    elif quantity == "density":
        if T > 0:
            def w(t):
                return 0.5 * (1.0 - np.tanh((a * np.cos(t) + b) / (2.0 * T)))
        else:
            def w(t):
                return 1.0 if a * np.cos(t) + b < 0 else 0.0
    else:
        raise ValueError(quantity)
    t0 = _theta(-b / a)
    cuts = sorted({lo, hi, min(max(t0, lo), hi)})
    c = np.zeros(N)
    for n in range(N):
        s = 0.0
        for p, q in zip(cuts[:-1], cuts[1:]):
            if q > p:
                if n == 0:
                    s += integrate.quad(w, p, q, limit=400, epsabs=1e-14, epsrel=1e-13)[0]
                else:
                    s += integrate.quad(w, p, q, weight="cos", wvar=n, limit=400, epsabs=1e-14)[0]
        c[n] = (1.0 if n == 0 else 2.0) / np.pi * s
    return c


def density(mu_ee, a, b, T=0.0, kernel="jackson", lam=0.0):
    """Electron density per site from the electron-density equation,
    n_i = int [N_up(E,i) + N_down(E,i)] f(E) dE with N_down = N_up (singlet
    pairing; the reading of the spin-down LDOS), i.e.
    n_i = 2 sum_n g_n c_n mu^ee_n(i) with c_n the coefficients of f(a x + b)."""
    mu_ee = np.asarray(mu_ee, dtype=np.float64)
    N = mu_ee.shape[-1]
    g = jackson(N) if kernel == "jackson" else lorentz(N, lam)
    return 2.0 * mu_ee @ (g * thermal_coefficients(N, a, b, T, quantity="density"))


def thermal_gap_weights(N, a, b, T, E_c=0.0, kernel="jackson", lam=0.0):
    """g_n c_n of eq. (op1) at temperature T (c_n of tanh(E/2T) on |E| < E_c)."""
    g = jackson(N) if kernel == "jackson" else lorentz(N, lam)
    return g * thermal_coefficients(N, a, b, T, E_c, "gap")


def gap_map_thermal(mu_he, U, a, b, T, E_c=0.0, kernel="jackson", lam=0.0, weights=None):
    """Eq. (op1) at temperature T: Delta_i = (U/2) conj(sum_n g_n c_n mu^he_n(i))
    with c_n the coefficients of tanh(E/2T) on |E| < E_c (reading of the
    prefactor as in gap_map).  weights: precomputed thermal_gap_weights."""
    mu_he = np.asarray(mu_he)
    N = mu_he.shape[-1]
    wts = thermal_gap_weights(N, a, b, T, E_c, kernel, lam) if weights is None else weights
    return 0.5 * np.asarray(U) * np.conj(mu_he @ wts)
