"""Pins for the oracle's scattering moments and efficiencies beyond Q_ext,
Q_abs, Q_sca: Q_pha, Q_bk, Q_sca g, <cos theta>, <cos^2 theta> and Q_pr
(guide, sections "What Does It Calculate?", "Calculation of <cos theta>,
Radiative Force, and Radiation Torque" and "Averaging over Scattering
Directions"), by the Mie series, its Rayleigh limit, a single dipole's
closed forms and the exact double sum for Q_sca."""
import numpy as np
import pytest

import synth
from oracle import dda, mie, scatter


def _mie_phase_moments(m, x, nth=40001):
    """<cos theta>, <cos^2 theta> of the Mie phase function by direct
    numerical integration over theta (unpolarized incidence)."""
    th = np.linspace(0.0, np.pi, nth)
    S1, S2 = mie.mie_amplitudes(m, x, th)
    p = 0.5 * (np.abs(S1) ** 2 + np.abs(S2) ** 2) * np.sin(th)
    z = np.trapezoid(p, th)
    return np.trapezoid(p * np.cos(th), th) / z, np.trapezoid(p * np.cos(th) ** 2, th) / z


@pytest.mark.parametrize("m,x", [(1.33 + 0.01j, 1.0), (1.5 + 0.1j, 3.0), (2.0 + 1.0j, 2.0)])
def test_mie_asymmetry_series_matches_integration(m, x):
    g_int, _ = _mie_phase_moments(m, x)
    assert abs(mie.mie_asymmetry(m, x) - g_int) < 1e-7


@pytest.mark.parametrize("m", [1.3 + 0.0j, 1.5 + 0.2j, 2.0 + 1.0j])
def test_mie_rayleigh_limits(m):
    """x -> 0: Q_pha -> 2x Re K, Q_bk -> x^4 |K|^2 / pi, <cos> -> 0, with
    K = (m^2 - 1)/(m^2 + 2) (a dipole of polarizability a^3 K)."""
    x = 1e-3
    K = (m * m - 1) / (m * m + 2)
    assert abs(mie.mie_phase_lag(m, x) / (2 * x * K.real) - 1) < 1e-5
    assert abs(mie.mie_backscatter(m, x) / (x ** 4 * abs(K) ** 2 / np.pi) - 1) < 1e-5
    assert abs(mie.mie_asymmetry(m, 0.01)) < 1e-3


def _single_dipole(kd=0.2, m=1.5 + 0.1j):
    r = np.zeros((1, 3))
    comp = np.array([1])
    kh, e, L = dda.waves_for_orientation(0.3, 0.8, 1.2)
    ainv = dda.site_inverse_polarizability(comp, [m], kd, dda.ALPHA_CM_RR)
    E = dda.incident_field(r, kd, kh, e[0])
    P = E / ainv[:, None]
    return r, kd, E, P, ainv, kh, L


def test_single_dipole_closed_forms():
    """N = 1: C_pha = 2 pi k Re(alpha), dC/dOmega(-khat) = k^4 |alpha|^2 (the
    dipole is transverse to khat), and the quadrature moments of the dipole
    pattern 1 - (n . e)^2: <cos theta> = 0, <cos^2 theta> = 2/5 (to the
    quadrature's accuracy)."""
    r, k, E, P, ainv, kh, L = _single_dipole()
    alpha = 1.0 / ainv[0]
    n_tf, w = scatter.quadrature_directions_tf(x=k * dda.effective_radius(1), eta=0.25, lab_axes=L)
    mo = scatter.scattering_moments(r, k, E, P, ainv, kh, n_tf, w)
    area = np.pi * dda.effective_radius(1) ** 2
    assert abs(mo["Qpha"] - 2 * np.pi * k * alpha.real / area) < 1e-14
    assert abs(mo["Qbk"] / (k ** 4 * abs(alpha) ** 2 / area) - 1) < 1e-12
    assert abs(mo["cos"]) < 2e-3
    assert abs(mo["cos2"] - 0.4) < 5e-3
    # Q_pr = Q_ext khat - Q_sca g
    assert np.allclose(mo["Qpr"], mo["Qext"] * kh - mo["Qsca_g"], atol=1e-15)


def test_quadrature_converges_to_the_double_sum():
    occ = synth.ellipsoid_occupancy((6, 6, 5), (5.6, 5.1, 4.3))
    r, comp, _ = dda.sites_from_occupancy(occ)
    m, k = [1.7 + 0.05j], 0.6
    kh, e, L = dda.waves_for_orientation(0.5, 1.0, 0.2)
    ainv = dda.site_inverse_polarizability(comp, m, k, dda.ALPHA_LDR, kh, e[0])
    E = dda.incident_field(r, k, kh, e[0])
    P = dda.solve_dense(r, k, ainv, E)
    exact = dda.scattering_double_sum(r, k, P)
    x = k * dda.effective_radius(len(r))
    errs = []
    for eta in (1.0, 0.5, 0.25):
        n_tf, w = scatter.quadrature_directions_tf(x, eta, L)
        errs.append(abs(scatter.scattering_moments(r, k, E, P, ainv, kh, n_tf, w)["Qsca_quad"] / exact - 1))
    assert errs[-1] < 2e-3 and errs[-1] < errs[0], errs


def test_sphere_moments_match_mie():
    """C1 sphere (D = 16, N = 2176, m = 1.33 + 0.01i, x = 1, LDR): the DDA
    values agree with Mie to the discretization error of this lattice."""
    occ = synth.sphere_occupancy(16)
    r, comp, _ = dda.sites_from_occupancy(occ)
    m, x = 1.33 + 0.01j, 1.0
    k = x / dda.effective_radius(len(r))
    kh, e, L = dda.waves_for_orientation(0.0, 0.0, 0.0)
    ainv = dda.site_inverse_polarizability(comp, [m], k, dda.ALPHA_LDR, kh, e[0])
    E = dda.incident_field(r, k, kh, e[0])
    P, _ = dda.solve_iterative(r, k, ainv, E, tol=1e-10)
    n_tf, w = scatter.quadrature_directions_tf(x, 0.5, L)
    mo = scatter.scattering_moments(r, k, E, P, ainv, kh, n_tf, w)
    g_mie, c2_mie = _mie_phase_moments(m, x)
    assert abs(mo["Qpha"] / mie.mie_phase_lag(m, x) - 1) < 5e-3
    assert abs(mo["Qbk"] / mie.mie_backscatter(m, x) - 1) < 2e-2
    assert abs(mo["cos"] - g_mie) < 3e-3
    assert abs(mo["cos2"] - c2_mie) < 1e-2
