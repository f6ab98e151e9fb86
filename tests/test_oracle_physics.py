"""Pins for the oracle's DDA physics: polarizability, interaction matrix,
solves, cross sections and amplitudes, each checked against something other
than the oracle itself (closed forms, brute force, identities, Mie theory)."""
import numpy as np
import pytest

import synth
from oracle import dda, mie, scatter

TWO_PI = 2 * np.pi


def _dipole_field(p, rvec, k):
    """Field at rvec of a point dipole p at the origin, written with cross
    products (Jackson-style vector form, Gaussian units):
        E = e^{ikr} { k^2 (n x p) x n / r + [3 n (n.p) - p] (1/r^3 - i k / r^2) }.
    Independent of the oracle's tensor form."""
    r = np.linalg.norm(rvec)
    n = rvec / r
    far = np.cross(np.cross(n, p), n) * k ** 2 / r
    near = (3 * n * np.dot(n, p) - p) * (1 / r ** 3 - 1j * k / r ** 2)
    return np.exp(1j * k * r) * (far + near)


def test_single_dipole_closed_form():
    """N = 1: P = alpha E, C_ext = 4 pi k Im(alpha), C_sca = (8 pi / 3) k^4 |alpha|^2."""
    k, m = 0.3, 1.5 + 0.2j
    r = np.zeros((1, 3))
    khat, e = np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
    ainv = np.array([dda.inverse_polarizability(m, k, dda.ALPHA_LDR, khat, e)])
    E = dda.incident_field(r, k, khat, e)
    P = dda.solve_dense(r, k, ainv, E)
    alpha = 1 / ainv[0]
    assert np.allclose(P, alpha * E)
    area = np.pi * dda.effective_radius(1) ** 2
    qext, qabs, qsca = dda.cross_sections(k, E, P, ainv)
    assert np.isclose(qext * area, 4 * np.pi * k * alpha.imag, rtol=1e-13)
    assert np.isclose(qsca * area, 8 * np.pi / 3 * k ** 4 * abs(alpha) ** 2, rtol=1e-12)
    assert np.isclose(dda.scattering_double_sum(r, k, P) * area, 8 * np.pi / 3 * k ** 4 * abs(alpha) ** 2)


@pytest.mark.parametrize("m", [1.33 + 0.01j, 1.7 + 0.1j, 2 + 1j])
def test_rayleigh_limit(m):
    """A single CM dipole with radiative reaction reaches the Rayleigh limit:
    Q_abs -> 4 x Im K, Q_sca -> (8/3) x^4 |K|^2, K = (eps-1)/(eps+2)."""
    K = (m ** 2 - 1) / (m ** 2 + 2)
    for x in [1e-3, 1e-2]:
        k = x / dda.effective_radius(1)
        r = np.zeros((1, 3))
        ainv = np.array([dda.inverse_polarizability(m, k, dda.ALPHA_CM_RR)])
        E = dda.incident_field(r, k, [1, 0, 0], [0, 0, 1])
        P = dda.solve_dense(r, k, ainv, E)
        qext, qabs, qsca = dda.cross_sections(k, E, P, ainv)
        assert np.isclose(qabs, 4 * x * K.imag, rtol=5 * x)
        assert np.isclose(qsca, 8 / 3 * x ** 4 * abs(K) ** 2, rtol=5 * x)
    # the same with the LDR prescription reduces to CM as k d -> 0
    for kd in [1e-3, 1e-4]:
        a_ldr = dda.inverse_polarizability(m, kd, dda.ALPHA_LDR, [1, 0, 0], [0, 1, 0])
        a_cm = dda.inverse_polarizability(m, kd, dda.ALPHA_CM)
        assert abs(a_ldr - a_cm) / abs(a_cm) < 10 * kd ** 2


def test_two_dipoles_brute_force():
    """N = 2 by self-consistent iteration with the vector dipole-field formula."""
    k, m = 0.7, 1.4 + 0.05j
    r = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, -1.5]])
    khat = np.array([0.6, 0.0, 0.8])
    e = np.array([0.8, 0.3j, -0.6]) / np.sqrt(1.09)
    alpha = 1 / dda.inverse_polarizability(m, k, dda.ALPHA_CM_RR)
    Einc = [e * np.exp(1j * k * np.dot(khat, rj)) for rj in r]
    P = [alpha * Einc[0], alpha * Einc[1]]
    for _ in range(200):
        P = [alpha * (Einc[0] + _dipole_field(P[1], r[0] - r[1], k)),
             alpha * (Einc[1] + _dipole_field(P[0], r[1] - r[0], k))]
    ainv = np.full(2, 1 / alpha)
    Pd = dda.solve_dense(r, k, ainv, np.stack(Einc))
    assert np.allclose(Pd, np.stack(P), rtol=1e-12, atol=1e-14)


def _cube8(two_materials):
    """The guide's 8-dipole demo cube (FROM_FILE examples), optionally with
    composition 2 on the JX = 1 half."""
    occ = np.ones((2, 2, 2), dtype=np.uint8)
    if two_materials:
        occ[:, :, 1] = 2
    return occ


@pytest.mark.parametrize("two", [False, True])
def test_matrix_symmetric_and_matvecs_agree(two):
    """A = A^T exactly; the C direct matvec equals the dense product."""
    occ = _cube8(two)
    r, comp, _ = dda.sites_from_occupancy(occ)
    assert np.allclose(r.mean(0), 0) and len(r) == 8
    k = 0.4
    ainv = dda.site_inverse_polarizability(comp, [1.5 + 0.01j, 2.0 + 1.0j], k, dda.ALPHA_LDR, [0, 0, 1], [1, 0, 0])
    A = dda.dense_matrix(r, k, ainv)
    assert np.max(np.abs(A - A.T)) == 0.0
    x = np.random.default_rng(0).standard_normal((8, 3)) + 1j * np.random.default_rng(1).standard_normal((8, 3))
    assert np.allclose(dda.matvec_direct(r, k, ainv, x).reshape(-1), A @ x.reshape(-1), rtol=1e-13, atol=1e-13)
    rows = np.array([5, 0, 7])
    assert np.allclose(dda.matvec_rows(r, k, ainv, x, rows), (A @ x.reshape(-1)).reshape(8, 3)[rows])


def _sphere_problem(D, m, x, kind=dda.ALPHA_LDR, beta=0.0, theta=0.0, phi=0.0):
    occ = synth.sphere_occupancy(D)
    r, comp, _ = dda.sites_from_occupancy(occ)
    k = x / dda.effective_radius(len(r))
    khat, es, L = dda.waves_for_orientation(beta, theta, phi)
    out = []
    for e in es:
        ainv = dda.site_inverse_polarizability(comp, [m], k, kind, khat, e)
        E = dda.incident_field(r, k, khat, e)
        out.append((ainv, E))
    return r, k, khat, es, L, out


def test_lu_and_bicgstab_agree():
    r, k, khat, es, L, probs = _sphere_problem(8, 1.5 + 0.1j, 2.0, theta=0.7, phi=0.3, beta=1.1)
    for ainv, E in probs:
        Pd = dda.solve_dense(r, k, ainv, E)
        Pi, info = dda.solve_iterative(r, k, ainv, E, tol=1e-11)
        assert info["rel_resid"] < 1e-11
        assert np.linalg.norm(Pd - Pi) / np.linalg.norm(Pd) < 1e-9
        rel, errtol = dda.residual_norms(r, k, ainv, E, Pd)
        assert rel < 1e-12 and errtol < 1e-10


def test_optical_theorem_three_routes():
    """Q_ext - Q_abs equals the exact pair double sum (to solve accuracy) and
    the angular quadrature of the far field (to quadrature accuracy)."""
    r, k, khat, es, L, probs = _sphere_problem(8, 1.33 + 0.01j, 3.0, theta=0.4, beta=0.2)
    for ainv, E in probs:
        P = dda.solve_dense(r, k, ainv, E)
        qext, qabs, qsca = dda.cross_sections(k, E, P, ainv)
        q2 = dda.scattering_double_sum(r, k, P)
        assert abs(q2 - qsca) / qsca < 1e-10
        q3 = scatter.scattering_quadrature(r, k, P, L, 3.0, eta=0.3)
        assert abs(q3 - qsca) / qsca < 1e-2


def test_forward_scattering_identity():
    """C_ext = (4 pi / k^2) Re S_2(0) for e01 = y (optical theorem in f_ml form),
    and likewise Re S_1(0) for the second polarization."""
    x = 2.0
    r, k, khat, es, L, probs = _sphere_problem(6, 1.6 + 0.3j, x, theta=0.9, phi=0.4, beta=0.5)
    Ps, qs = [], []
    for ainv, E in probs:
        P = dda.solve_dense(r, k, ainv, E)
        Ps.append(P)
        qs.append(dda.cross_sections(k, E, P, ainv)[0])
    f = scatter.scattering_amplitudes(r, k, Ps, np.array([0.0]), np.array([0.0]), L)
    e01, e02 = dda.incident_polarizations((0, 1, 0))
    S = scatter.amplitude_matrix(f, np.array([0.0]), e01, e02)
    area = np.pi * dda.effective_radius(len(r)) ** 2
    assert np.isclose(4 * np.pi / k ** 2 * S[0, 1].real / area, qs[0], rtol=1e-12)
    assert np.isclose(4 * np.pi / k ** 2 * S[0, 0].real / area, qs[1], rtol=1e-12)


@pytest.mark.slow
def test_dda_converges_to_mie():
    """At fixed x = 1, m = 1.33+0.01i the DDA pseudosphere approaches Mie as
    the lattice is refined (guide: 'few percent' accuracy for |m| k d < 1), and
    the amplitude functions agree in both scattering planes."""
    m, x = 1.33 + 0.01j, 1.0
    qm = np.array(mie.mie_efficiencies(m, x))
    errs = []
    for D in (6, 10, 16):
        r, k, khat, es, L, probs = _sphere_problem(D, m, x)
        ainv, E = probs[0]
        P, info = dda.solve_iterative(r, k, ainv, E, tol=1e-10)
        q = np.array(dda.cross_sections(k, E, P, ainv))
        errs.append(np.abs(q - qm) / qm)
    errs = np.array(errs)
    assert np.all(np.diff(errs[:, 0]) < 0) and np.all(np.diff(errs[:, 2]) < 0)
    assert errs[-1, 0] < 0.02 and errs[-1, 2] < 0.02 and errs[-1, 1] < 0.05
    # S_1, S_2 at D = 16 against Mie in the phi = 0 and phi = 90 deg planes
    r, k, khat, es, L, probs = _sphere_problem(16, m, x)
    Ps = [dda.solve_iterative(r, k, a, E, tol=1e-10)[0] for a, E in probs]
    th = np.deg2rad(np.arange(0, 181, 5.0))
    S1m, S2m = mie.mie_amplitudes(m, x, th)
    e01, e02 = dda.incident_polarizations((0, 1, 0))
    for phi in (0.0, np.pi / 2):
        ph = np.full_like(th, phi)
        f = scatter.scattering_amplitudes(r, k, Ps, th, ph, L)
        S = scatter.amplitude_matrix(f, ph, e01, e02)
        assert np.max(np.abs(S[:, 0] - S1m)) / np.max(np.abs(S1m)) < 0.03
        assert np.max(np.abs(S[:, 1] - S2m)) / np.max(np.abs(S1m)) < 0.03
        assert np.max(np.abs(S[:, 2:])) / np.max(np.abs(S1m)) < 1e-3


def test_cabs_of_lossless_target_vanishes():
    """For real m, CM/LDR give Im(1/alpha) = -(2/3) k^3 exactly, so Q_abs = 0."""
    r, k, khat, es, L, probs = _sphere_problem(6, 1.5 + 0j, 2.0)
    ainv, E = probs[0]
    P = dda.solve_dense(r, k, ainv, E)
    qext, qabs, qsca = dda.cross_sections(k, E, P, ainv)
    assert abs(qabs) < 1e-12 * qext


def test_shifted_guess_exact_for_isolated_dipole():
    """One dipole off the origin, incidence rotated about a fixed polarization:
    the exact new solution alpha_new E_inc,new(r0) is reproduced, with LDR
    polarizabilities that differ between the two directions (S = 0 vs 8/25)."""
    k, m = 0.4, 1.5 + 0.1j
    r = np.array([[0.3, -1.2, 2.1]])
    e = np.array([1.0, 2.0, 0.0]) / np.sqrt(5)
    kp, kn = np.array([0.0, 0.0, 1.0]), np.array([2.0, -1.0, 0.0]) / np.sqrt(5)
    ap = np.array([dda.inverse_polarizability(m, k, dda.ALPHA_LDR, kp, e)])
    an = np.array([dda.inverse_polarizability(m, k, dda.ALPHA_LDR, kn, e)])
    assert abs(ap[0] - an[0]) > 1e-3 * abs(an[0])
    Pp = dda.incident_field(r, k, kp, e) / ap[:, None]
    e_sh, P0 = dda.shifted_previous_guess(r, k, Pp, ap, an, kp, kn)
    En = dda.incident_field(r, k, kn, e)
    assert np.allclose(e_sh, En, rtol=1e-14)
    assert np.allclose(P0, En / an[:, None], rtol=1e-14)


def test_shifted_guess_same_wave_and_static_limit():
    """Same wave twice: the guess is the previous solution.  Static limit
    (k -> 0) with the polarization kept: the local field no longer depends on
    the incidence direction, so the shifted guess solves the new system to O(k)."""
    occ = synth.sphere_occupancy(6)
    r, comp, _ = dda.sites_from_occupancy(occ)
    m = 1.6 + 0.2j
    e = np.array([0.0, 0.0, 1.0])
    kp, kn = np.array([1.0, 0.0, 0.0]), np.array([0.6, 0.8, 0.0])
    for k, bound in ((0.5, None), (1e-4, 1e-3)):
        ainv = np.full(len(r), dda.inverse_polarizability(m, k, dda.ALPHA_CM_RR))
        Pp = dda.solve_dense(r, k, ainv, dda.incident_field(r, k, kp, e))
        _, same = dda.shifted_previous_guess(r, k, Pp, ainv, ainv, kp, kp)
        assert np.allclose(same, Pp, rtol=1e-14, atol=0)
        if bound is None:
            continue
        _, P0 = dda.shifted_previous_guess(r, k, Pp, ainv, ainv, kp, kn)
        En = dda.incident_field(r, k, kn, e)
        rel = np.linalg.norm(En.reshape(-1) - dda.dense_matrix(r, k, ainv) @ P0.reshape(-1)) / np.linalg.norm(En)
        assert rel < bound


def test_projected_guess_recovers_solution_in_span_and_is_optimal():
    """If the history holds the new wave's own solution the projection returns
    it; with one basis vector the coefficient is the closed form <w,E>/<w,w>;
    the projection's residual is never above that of any single basis vector."""
    occ = synth.ellipsoid_occupancy((5, 6, 4), (5.0, 6.0, 4.0))
    r, comp, _ = dda.sites_from_occupancy(occ)
    k, m = 0.7, [1.4 + 0.1j]
    waves = [dda.waves_for_orientation(0.2, th, 0.5) for th in (0.6, 0.75, 0.9, 1.05)]
    sols = []
    for kh, es, _ in waves:
        a = dda.site_inverse_polarizability(comp, m, k, dda.ALPHA_LDR, kh, es[0])
        sols.append((dda.solve_dense(r, k, a, dda.incident_field(r, k, kh, es[0])), a, kh))
    kn, en, _ = waves[3]
    an = sols[3][1]
    En = dda.incident_field(r, k, kn, en[0])

    def res(P0):
        return np.linalg.norm(En - dda.matvec_direct(r, k, an, P0)) / np.linalg.norm(En)

    P0, c = dda.projected_history_guess(r, k, an, kn, En, sols[:3] + [sols[3]])
    assert res(P0) < 1e-10 and abs(c[3] - 1) < 1e-8
    P1, c1 = dda.projected_history_guess(r, k, an, kn, En, sols[2:3])
    _, v = dda.shifted_previous_guess(r, k, *sols[2][:2], an, sols[2][2], kn)
    w = dda.matvec_direct(r, k, an, v).reshape(-1)
    assert np.isclose(c1[0], np.vdot(w, En.reshape(-1)) / np.vdot(w, w), rtol=1e-10)
    P3, _ = dda.projected_history_guess(r, k, an, kn, En, sols[:3])
    for P, a, kh in sols[:3]:
        _, v = dda.shifted_previous_guess(r, k, P, a, an, kh, kn)
        assert res(P3) <= res(v) + 1e-14
    assert res(P3) < res(P1)
