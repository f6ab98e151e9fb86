"""Pins of the polarized differential cross sections (oracle/scatter.py
polarized_cross_sections) against the scattered field itself: with the
amplitude matrix, E_s is proportional to [[S2, S3], [S4, S1]] E_i in the
(parallel, perpendicular) basis (Bohren & Huffman, the convention of the
guide's Mueller elements), so dC_sca/dOmega of each scattered component is
|E_s,comp|^2 / k^2 per unit incident intensity.  The incident Stokes vector
follows the same book: I = |E_par|^2 + |E_perp|^2, Q = |E_par|^2 -
|E_perp|^2, U = 2 Re(E_par E_perp^*), V = -2 Im(E_par E_perp^*)."""
import numpy as np
import pytest

from oracle import scatter


def _stokes(e):
    ep, es = e
    return np.array([abs(ep) ** 2 + abs(es) ** 2, abs(ep) ** 2 - abs(es) ** 2,
                     2 * np.real(ep * np.conj(es)), -2 * np.imag(ep * np.conj(es))])


def _direct(S, e, k):
    S1, S2, S3, S4 = S
    par = S2 * e[0] + S3 * e[1]
    perp = S4 * e[0] + S1 * e[1]
    n = abs(e[0]) ** 2 + abs(e[1]) ** 2
    return np.array([abs(par) ** 2, abs(perp) ** 2, abs(par) ** 2 + abs(perp) ** 2]) / (k * k * n)


@pytest.mark.parametrize("seed", range(6))
def test_polarized_cross_sections_equal_the_scattered_field(seed):
    rng = np.random.default_rng(seed)
    S = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    M = scatter.mueller(S)
    k = 0.3 + rng.random()
    # linear at several angles, the two circular states and a random elliptical one
    states = [np.array([np.cos(g), np.sin(g)], complex) for g in (0.0, np.pi / 2, 0.37, 1.9)]
    states += [np.array([1, 1j]) / np.sqrt(2), np.array([1, -1j]) / np.sqrt(2)]
    states += [rng.standard_normal(2) + 1j * rng.standard_normal(2)]
    for e in states:
        got = scatter.polarized_cross_sections(M, k, _stokes(e))
        assert np.allclose(got, _direct(S, e, k), rtol=1e-12, atol=1e-15), e


def test_unpolarized_incidence_is_the_mean_of_two_orthogonal_states():
    rng = np.random.default_rng(7)
    S = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    M = scatter.mueller(S)
    k = 0.8
    un = scatter.polarized_cross_sections(M, k, [1, 0, 0, 0])
    a = _direct(S, np.array([1, 0], complex), k)
    b = _direct(S, np.array([0, 1], complex), k)
    assert np.allclose(un, 0.5 * (a + b), rtol=1e-12)
    # and the guide's forms: (|S2|^2 + |S3|^2) / 2k^2, (|S1|^2 + |S4|^2) / 2k^2, S11 / k^2
    S1, S2, S3, S4 = S
    assert np.allclose(un, [(abs(S2) ** 2 + abs(S3) ** 2) / (2 * k * k), (abs(S1) ** 2 + abs(S4) ** 2) / (2 * k * k),
                            M[0, 0] / k ** 2], rtol=1e-12)


def test_dipole_at_right_angles_is_fully_polarized():
    # a point dipole: S1 constant, S2 = S1 cos(theta), S3 = S4 = 0; at 90 degrees P = 1
    for th in (np.pi / 2, 1.2, 0.4):
        S = np.array([0.3 + 0.2j, (0.3 + 0.2j) * np.cos(th), 0, 0])
        P = scatter.linear_polarization(scatter.mueller(S))
        assert P == pytest.approx(np.sin(th) ** 2 / (1 + np.cos(th) ** 2), rel=1e-12)
