"""Pins for the oracle's orientational sampling, averaging weights and the
combination of two polarization solutions into other target rotations Phi
(guide, sections "Sampling in Theta, Phi, and beta", "Orientational
Averaging" and the IORTH remark of "Scattering by Finite Targets")."""
import os

import numpy as np
import pytest

import synth
from oracle import dda
from oracle import orient as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "orientation_sampling.txt")


def _golden():
    out = []
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if not line:
            continue
        head, vals = line.split("|")
        name, lo, hi, n = head.split()
        out.append((name, float(lo), float(hi), int(n), [float(v) for v in vals.split()]))
    return out


@pytest.mark.parametrize("name,lo,hi,n,want", _golden())
def test_printed_sampling_examples(name, lo, hi, n, want):
    lo, hi = np.deg2rad(lo), np.deg2rad(hi)
    got = O.theta_samples(lo, hi, n) if name == "theta" else O.midpoints(lo, hi, n)
    # beta and Phi ascend; Theta follows cos(Theta) from cos(lo) to cos(hi)
    assert np.allclose(np.sort(np.rad2deg(got)), want, atol=0.006), (name, np.rad2deg(got))


def test_even_theta_cosines_are_interval_midpoints():
    assert np.allclose(np.sort(np.cos(O.theta_samples(0.0, np.pi / 2, 2))), [0.25, 0.75])


@pytest.mark.parametrize("counts", [(1, 1, 1), (2, 3, 2), (3, 5, 4), (4, 2, 3), (1, 7, 1), (5, 4, 6)])
def test_weights_sum_to_one(counts):
    _, _, _, w = O.orientation_samples(np.deg2rad([0, 360, 0, 180, 0, 360]), counts)
    assert w.shape == counts and abs(w.sum() - 1.0) < 1e-14 and (w > 0).all()


@pytest.mark.parametrize("nt", [3, 5, 7, 9])
def test_simpson_in_cos_theta_is_exact_for_cubics(nt):
    """Odd NTHETA over [0, pi]: the weighted sum of a cubic in cos(Theta) equals
    its mean over [-1, 1], (1/2) int p(u) du, computed from the antiderivative."""
    rng = np.random.default_rng(nt)
    a = rng.standard_normal(4)
    th = O.theta_samples(0.0, np.pi, nt)
    u = np.cos(th)
    got = np.sum(O.theta_weights(nt) * (a[0] + a[1] * u + a[2] * u ** 2 + a[3] * u ** 3))
    want = 0.5 * (2 * a[0] + 2 * a[2] / 3.0)  # odd powers integrate to zero
    assert abs(got - want) < 1e-13


@pytest.mark.parametrize("nt", [2, 4, 6])
def test_even_theta_average_is_exact_for_lines(nt):
    th = O.theta_samples(0.3, 2.1, nt)
    u = np.cos(th)
    got = np.sum(O.theta_weights(nt) * (2.0 - 3.0 * u))
    want = 2.0 - 3.0 * 0.5 * (np.cos(0.3) + np.cos(2.1))
    assert abs(got - want) < 1e-13


def test_random_orientation_averages_of_the_frame():
    """Over beta, Phi in [0, 2 pi) and Theta in [0, pi] every squared
    coefficient of a lab axis on a target axis averages to 1/3 (the lab axes
    are uniformly distributed directions); the sampling integrates these
    trigonometric polynomials exactly (NBETA, NPHI >= 3, odd NTHETA)."""
    b, t, p, w = O.orientation_samples(np.deg2rad([0, 360, 0, 180, 0, 360]), (4, 5, 4))
    sq = np.empty((len(b), len(t), len(p), 3, 3))
    for i, be in enumerate(b):
        for j, th in enumerate(t):
            for k, ph in enumerate(p):
                sq[i, j, k] = dda.lab_axes_in_target_frame(be, th, ph) ** 2
    avg = O.orientational_average(sq, w)
    assert np.allclose(avg, 1.0 / 3.0, atol=1e-13), avg


def test_phi_coefficients_are_a_rotation_and_khat_is_shared():
    rng = np.random.default_rng(5)
    for _ in range(5):
        be, th, p0, p1 = rng.uniform(0, 2 * np.pi, 4)
        c = O.phi_coefficients(be, th, p0, p1)
        assert np.allclose(c @ np.conj(c).T, np.eye(2), atol=1e-13)
        k0, _, _ = dda.waves_for_orientation(be, th, p0)
        k1, _, _ = dda.waves_for_orientation(be, th, p1)
        assert np.allclose(k0, k1, atol=1e-13)


def _blob(seed=3):
    occ = synth.ellipsoid_occupancy((6, 5, 5), (5.5, 4.2, 3.6))
    r, comp, _ = dda.sites_from_occupancy(occ)
    return r, comp


@pytest.mark.parametrize("kind", [dda.ALPHA_CM, dda.ALPHA_CM_RR])
def test_phi_combination_matches_direct_solves(kind):
    """With a polarization-independent polarizability the combined pair equals
    the solutions computed directly at the rotated orientation."""
    r, comp = _blob()
    m, k = [1.6 + 0.2j], 0.7
    be, th, p0 = 0.4, 1.1, 0.2
    kh0, e0, _ = dda.waves_for_orientation(be, th, p0)
    ainv = dda.site_inverse_polarizability(comp, m, k, kind)
    E0 = np.stack([dda.incident_field(r, k, kh0, e0[l]) for l in range(2)])
    P0 = np.stack([dda.solve_dense(r, k, ainv, E0[l]) for l in range(2)])
    for p1 in (0.9, 2.5, 4.0):
        kh1, e1, _ = dda.waves_for_orientation(be, th, p1)
        c = O.phi_coefficients(be, th, p0, p1)
        Pc = O.combine_pair(c, P0)
        for l in range(2):
            E1 = dda.incident_field(r, k, kh1, e1[l])
            P1 = dda.solve_dense(r, k, ainv, E1)
            assert np.linalg.norm(Pc[l] - P1) < 1e-11 * np.linalg.norm(P1)
            q_direct = dda.cross_sections(k, E1, P1, ainv)
            q_comb = O.cross_sections_at_phi(k, E0, P0, ainv, c)[l]
            assert np.allclose(q_comb, q_direct, rtol=1e-11, atol=1e-14)


def test_phi_combination_is_approximate_for_ldr():
    """LDR's 1/alpha depends on the polarization through S, so the combination
    misses the rotated solution, by a small but nonzero amount."""
    r, comp = _blob()
    m, k = [1.6 + 0.2j], 0.7
    be, th, p0, p1 = 0.4, 1.1, 0.2, 1.3
    kh0, e0, _ = dda.waves_for_orientation(be, th, p0)
    kh1, e1, _ = dda.waves_for_orientation(be, th, p1)
    P0 = []
    for l in range(2):
        ai = dda.site_inverse_polarizability(comp, m, k, dda.ALPHA_LDR, kh0, e0[l])
        P0.append(dda.solve_dense(r, k, ai, dda.incident_field(r, k, kh0, e0[l])))
    c = O.phi_coefficients(be, th, p0, p1)
    Pc = O.combine_pair(c, np.stack(P0))
    ai1 = dda.site_inverse_polarizability(comp, m, k, dda.ALPHA_LDR, kh1, e1[0])
    P1 = dda.solve_dense(r, k, ai1, dda.incident_field(r, k, kh1, e1[0]))
    rel = np.linalg.norm(Pc[0] - P1) / np.linalg.norm(P1)
    assert 1e-8 < rel < 5e-2, rel
