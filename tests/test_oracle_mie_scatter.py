"""Pins for the oracle's Mie series, Mueller algebra and angular quadrature."""
import os

import numpy as np
import pytest

from oracle import mie, scatter

GOLD = os.path.join(os.path.dirname(__file__), "golden", "worked_example_mueller.txt")


@pytest.mark.parametrize("m", [1.33 + 0.01j, 2 + 1j, 1.5 + 0j])
def test_mie_rayleigh_limit(m):
    K = (m ** 2 - 1) / (m ** 2 + 2)
    x = 1e-3
    qext, qabs, qsca = mie.mie_efficiencies(m, x)
    assert np.isclose(qsca, 8 / 3 * x ** 4 * abs(K) ** 2, rtol=1e-4)
    if m.imag:
        assert np.isclose(qabs, 4 * x * K.imag, rtol=1e-3)


@pytest.mark.parametrize("m,x", [(1.33 + 0.01j, 1.0), (1.5 + 0.1j, 10.0), (2 + 1j, 7.0), (1.5 + 0j, 5.0)])
def test_mie_optical_theorem_and_phase_function(m, x):
    """Q_ext = 4 Re S(0) / x^2 and Q_sca = integral of (|S1|^2+|S2|^2)/2 dOmega / (pi x^2)."""
    qext, qabs, qsca = mie.mie_efficiencies(m, x)
    S1, S2 = mie.mie_amplitudes(m, x, np.array([0.0]))
    assert np.isclose(S1[0], S2[0])
    assert np.isclose(4 * S1[0].real / x ** 2, qext, rtol=1e-12)
    th = np.linspace(0, np.pi, 4001)
    S1, S2 = mie.mie_amplitudes(m, x, th)
    integrand = 0.5 * (np.abs(S1) ** 2 + np.abs(S2) ** 2) * np.sin(th)
    integral = 2 * np.pi * np.trapezoid(integrand, th)
    assert np.isclose(integral / (np.pi * x ** 2), qsca, rtol=1e-5)
    if m.imag == 0:
        assert abs(qabs) < 1e-12


def test_mie_large_sphere_extinction_paradox():
    """Q_ext -> 2 for a large absorbing sphere; the approach is from above with
    an edge term of order x^(-2/3)."""
    d = [mie.mie_efficiencies(1.5 + 0.5j, x)[0] - 2.0 for x in (300.0, 2000.0)]
    assert 0 < d[1] < d[0] and d[1] < 0.02


def test_mie_index_matched_sphere_is_invisible():
    qext, qabs, qsca = mie.mie_efficiencies(1.0 + 0j, 3.0)
    assert abs(qext) < 1e-14 and abs(qsca) < 1e-14


def _gold():
    rows = [list(map(float, l.split())) for l in open(GOLD) if l.strip() and not l.startswith("#")]
    return np.array(rows)


def test_printed_polarization_column():
    """The printed Pol. column equals (S21^2 + S31^2)^(1/2) / S11 of the printed
    elements (guide, definition of P), to the printed precision."""
    g = _gold()
    M = np.zeros((len(g), 4, 4))
    M[:, 0, 0], M[:, 1, 0], M[:, 2, 0] = g[:, 3], g[:, 5], g[:, 7]
    P = scatter.linear_polarization(M)
    assert np.allclose(P, g[:, 2], atol=2e-4 + 2e-3 * g[:, 2])


def test_mueller_relations_for_symmetric_target():
    """With S3 = S4 = 0 (a target with the worked example's symmetry) the
    bilinears give S12 = S21, S22 = S11, S31 = S41 = 0, as in the printed
    table; and general identities hold for random amplitudes."""
    rng = np.random.default_rng(3)
    S = rng.standard_normal((20, 4)) + 1j * rng.standard_normal((20, 4))
    S[:, 2:] = 0
    M = scatter.mueller(S)
    assert np.allclose(M[:, 0, 1], M[:, 1, 0]) and np.allclose(M[:, 1, 1], M[:, 0, 0])
    assert np.allclose(M[:, 2, 0], 0) and np.allclose(M[:, 3, 0], 0)
    g = _gold()
    assert np.allclose(g[:, 4], g[:, 5], rtol=2e-3, atol=1e-5)
    assert np.allclose(g[:, 3], g[:, 6], rtol=1e-3)
    # a Mueller matrix built from one amplitude matrix is "pure":
    # sum_ij S_ij^2 = 4 S_11^2 (Hovenier's identity), random S
    S = rng.standard_normal((20, 4)) + 1j * rng.standard_normal((20, 4))
    M = scatter.mueller(S)
    assert np.allclose(np.sum(M ** 2, axis=(1, 2)), 4 * M[:, 0, 0] ** 2)
    # relations printed in "Relation Between Mueller Matrix and Scattering
    # Cross Sections": unpolarized incidence, E_s parallel to the scattering
    # plane: (|S2|^2+|S3|^2)/2 = (S11+S21)/2; perpendicular: (S11-S21)/2;
    # incidence and detection parallel: |S2|^2 = (S11+S12+S21+S22)/2
    a = np.abs(S) ** 2
    assert np.allclose((a[:, 1] + a[:, 2]) / 2, (M[:, 0, 0] + M[:, 1, 0]) / 2)
    assert np.allclose((a[:, 0] + a[:, 3]) / 2, (M[:, 0, 0] - M[:, 1, 0]) / 2)
    assert np.allclose(a[:, 1], (M[:, 0, 0] + M[:, 0, 1] + M[:, 1, 0] + M[:, 1, 1]) / 2)


def test_amplitude_matrix_unit_cases():
    """e01 = y, e02 = z: at phi = 0, S2 = -i f11, S1 = -i f22, S3 = i f12,
    S4 = i f21; at phi = 90 deg the roles of the two lab axes swap."""
    rng = np.random.default_rng(5)
    f = rng.standard_normal((1, 2, 2)) + 1j * rng.standard_normal((1, 2, 2))
    S = scatter.amplitude_matrix(f, np.array([0.0]), [0, 1, 0], [0, 0, 1])[0]
    assert np.allclose(S, [-1j * f[0, 1, 1], -1j * f[0, 0, 0], 1j * f[0, 0, 1], 1j * f[0, 1, 0]])
    S = scatter.amplitude_matrix(f, np.array([np.pi / 2]), [0, 1, 0], [0, 0, 1])[0]
    assert np.allclose(S, [-1j * (-f[0, 1, 0]), -1j * f[0, 0, 1], 1j * (-f[0, 0, 0]), 1j * f[0, 1, 1]])


@pytest.mark.parametrize("x,eta", [(1.0, 1.0), (6.187304, 0.5), (20.0, 0.5)])
def test_quadrature_integrates_moments(x, eta):
    """Weights sum to 4 pi and integrate 1, cos, cos^2 close to 1, 0, 1/3."""
    th, ph, w = scatter.scattering_directions(x, eta)
    assert abs(w.sum() - 4 * np.pi) < 1e-12
    assert abs(np.sum(w * np.cos(th)) / (4 * np.pi)) < 1e-3
    # the guide reports angular-average errors of order 0.01 at eta = 1
    assert abs(np.sum(w * np.cos(th) ** 2) / (4 * np.pi) - 1 / 3) < 0.02 * eta
    grid = scatter.scattering_theta_grid(x, eta)
    assert grid[0] == 0 and np.isclose(grid[-1], np.pi) and np.all(np.diff(grid) > 0)
    # design rule: max spacing about eta (pi/2)/(3+x), attained near theta = pi
    dmax = np.max(np.diff(grid))
    assert 0.7 < dmax / (eta * (np.pi / 2) / (3 + x)) < 1.3


def test_quadrature_direction_count_matches_worked_example():
    """The worked example (x = 6.187304, ETASCA = 0.5) prints NAVG = 2292
    scattering directions used for Q_sca and g; the eta prescription with
    N_theta rounded to the nearest integer gives exactly that count."""
    th, ph, w = scatter.scattering_directions(6.187304, 0.5)
    assert len(th) == 2292
