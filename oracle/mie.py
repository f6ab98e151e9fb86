"""Oracle: Mie theory for a homogeneous sphere (test infrastructure only).

The guide validates the DDA against exact Mie results for spheres (figures
for m = 1.33+0.01i and m = 2+i in "Applicability of the DDA") and points to
Bohren & Huffman (1983) for the amplitude-matrix conventions.  This is the
standard Lorenz-Mie series in the Bohren & Huffman notation, written from the
textbook mathematics:

* logarithmic derivative D_n(m x) by downward recurrence,
* Riccati-Bessel psi_n(x) and chi_n(x) by upward recurrence, xi_n = psi_n - i chi_n,
* a_n, b_n from D_n, psi_n, xi_n,
* Q_ext = (2/x^2) sum (2n+1) Re(a_n + b_n), Q_sca = (2/x^2) sum (2n+1)(|a_n|^2 + |b_n|^2),
* S_1, S_2 from the angular functions pi_n, tau_n.

Time dependence exp(-i omega t), as in the guide.
"""
from __future__ import annotations

import numpy as np


def mie_coefficients(m: complex, x: float, nstop: int | None = None):
    """(a_n, b_n) for n = 1..nstop."""
    m = complex(m)
    if nstop is None:
        nstop = int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    y = m * x
    nmx = int(max(nstop, abs(y))) + 16
    D = np.zeros(nmx + 1, dtype=np.complex128)
    for n in range(nmx, 0, -1):
        D[n - 1] = n / y - 1.0 / (D[n] + n / y)
    psi_m2, psi_m1 = np.cos(x), np.sin(x)    # psi_{-1}, psi_0
    chi_m2, chi_m1 = -np.sin(x), np.cos(x)   # chi_{-1}, chi_0
    xi_m1 = psi_m1 - 1j * chi_m1
    a = np.zeros(nstop, dtype=np.complex128)
    b = np.zeros(nstop, dtype=np.complex128)
    for n in range(1, nstop + 1):
        psi = (2 * n - 1) / x * psi_m1 - psi_m2
        chi = (2 * n - 1) / x * chi_m1 - chi_m2
        xi = psi - 1j * chi
        ta = D[n] / m + n / x
        tb = D[n] * m + n / x
        a[n - 1] = (ta * psi - psi_m1) / (ta * xi - xi_m1)
        b[n - 1] = (tb * psi - psi_m1) / (tb * xi - xi_m1)
        psi_m2, psi_m1 = psi_m1, psi
        chi_m2, chi_m1 = chi_m1, chi
        xi_m1 = xi
    return a, b


def mie_efficiencies(m: complex, x: float):
    """(Q_ext, Q_abs, Q_sca) for a sphere of size parameter x and index m."""
    a, b = mie_coefficients(m, x)
    n = np.arange(1, len(a) + 1)
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return float(qext), float(qext - qsca), float(qsca)


def mie_amplitudes(m: complex, x: float, theta):
    """(S_1(theta), S_2(theta)) for scattering angles theta (radians)."""
    a, b = mie_coefficients(m, x)
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    mu = np.cos(theta)
    S1 = np.zeros(theta.shape, dtype=np.complex128)
    S2 = np.zeros(theta.shape, dtype=np.complex128)
    pi_m1 = np.zeros_like(mu)  # pi_0
    pi_n = np.ones_like(mu)    # pi_1
    for n in range(1, len(a) + 1):
        tau_n = n * mu * pi_n - (n + 1) * pi_m1
        fn = (2 * n + 1) / (n * (n + 1))
        S1 += fn * (a[n - 1] * pi_n + b[n - 1] * tau_n)
        S2 += fn * (a[n - 1] * tau_n + b[n - 1] * pi_n)
        pi_next = ((2 * n + 1) * mu * pi_n - (n + 1) * pi_m1) / n
        pi_m1, pi_n = pi_n, pi_next
    return S1, S2


def mie_asymmetry(m: complex, x: float):
    """<cos theta> from the series Q_sca <cos theta> = (4/x^2) [sum n(n+2)/(n+1)
    Re(a_n a_{n+1}^* + b_n b_{n+1}^*) + sum (2n+1)/(n(n+1)) Re(a_n b_n^*)]
    (Bohren & Huffman, the asymmetry parameter of a sphere)."""
    a, b = mie_coefficients(m, x)
    n = np.arange(1, len(a) + 1)
    t1 = np.sum((n[:-1] * (n[:-1] + 2) / (n[:-1] + 1)) * np.real(a[:-1] * np.conj(a[1:]) + b[:-1] * np.conj(b[1:])))
    t2 = np.sum((2 * n + 1) / (n * (n + 1)) * np.real(a * np.conj(b)))
    _, _, qsca = mie_efficiencies(m, x)
    return float(4.0 / x ** 2 * (t1 + t2) / qsca)


def mie_backscatter(m: complex, x: float):
    """Q_bk = (dC_sca/dOmega at theta = pi) / (pi a^2) = |S_1(pi)|^2 / (pi x^2)."""
    S1, _ = mie_amplitudes(m, x, np.pi)
    return float(np.abs(S1[0]) ** 2 / (np.pi * x ** 2))


def mie_phase_lag(m: complex, x: float):
    """Q_pha = -(2/x^2) Im S(0): the forward amplitude's imaginary part (with
    the scattered field exp(ikr)/(-ikr) S E_0 a dipole of polarizability alpha
    has S(0) = -i k^3 alpha, and a dilute medium of such dipoles retards the
    phase by 2 pi k Re(alpha) per unit target column, so
    C_pha = -(2 pi / k^2) Im S(0))."""
    S1, _ = mie_amplitudes(m, x, 0.0)
    return float(-2.0 / x ** 2 * np.imag(S1[0]))
