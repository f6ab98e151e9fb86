"""Oracle pins for anisotropic materials (guide, "Composite Targets with
Anisotropic Constituents"): per composition three principal refractive
indices and the Dielectric Frame angles (Theta_DF, Phi_DF, beta_DF); the
polarizability is diagonal in that frame and a symmetric 3 x 3 tensor in
the target frame.

Pins: the frame is orthonormal and right-handed and reduces to the identity
and to a rotation about x by beta_DF; equal principal indices give the
isotropic 1/alpha times the identity for any angles; an isolated dipole
polarized along a principal axis responds with that axis's polarizability,
and its efficiencies satisfy the optical theorem only with the tensor form
of the absorption sum; the matrix stays complex symmetric; and a 90-degree
rotation of material, lattice and incident wave together rotates the
solution (a cube of sites, dense LU solves)."""
import numpy as np
import pytest

from oracle import dda

M3 = [1.58 + 0.03j, 1.30 + 0.01j, 1.30 + 0.01j]  # uniaxial: extraordinary along e_1


def test_dielectric_frame_is_a_rotation():
    for ang in [(0.0, 0.0, 0.0), (0.3, 0.5, 0.7), (2.0, -1.0, 4.0)]:
        F = dda.dielectric_frame(*ang)
        assert np.allclose(F @ F.T, np.eye(3), atol=1e-14)
        assert np.isclose(np.linalg.det(F), 1.0)
    assert np.allclose(dda.dielectric_frame(0, 0, 0), np.eye(3))
    b = 0.4  # Theta = Phi = 0: a rotation by beta about e_1 = x
    assert np.allclose(dda.dielectric_frame(0, 0, b), [[1, 0, 0], [0, np.cos(b), np.sin(b)], [0, -np.sin(b), np.cos(b)]])


@pytest.mark.parametrize("kind", [dda.ALPHA_CM, dda.ALPHA_CM_RR, dda.ALPHA_LDR])
def test_equal_principal_indices_are_isotropic(kind):
    m, k = 1.5 + 0.1j, 0.4
    kh, e = np.array([0.0, 0.6, 0.8]), np.array([1.0, 0.0, 0.0])
    T = dda.anisotropic_inverse_polarizability([m, m, m], (0.7, -0.3, 1.9), k, kind, kh, e)
    assert np.allclose(T, dda.inverse_polarizability(m, k, kind, kh, e) * np.eye(3), atol=1e-13)
    assert np.allclose(T, T.T)


def test_single_dipole_principal_response_and_optical_theorem():
    """N = 1: P = alpha E.  E along e_j gives P = alpha_j E; for any E the
    radiative-reaction prescription makes C_ext = C_abs + C_sca with
    C_sca = (8 pi / 3) k^4 |P|^2 exactly, with the tensor absorption sum."""
    k = 0.3
    ang = (0.9, 0.4, -1.2)
    F = dda.dielectric_frame(*ang)
    kh = np.array([0.0, 0.0, 1.0])
    r = np.zeros((1, 3))
    for j in range(3):
        e = F[j].astype(np.complex128)
        T = dda.anisotropic_inverse_polarizability(M3, ang, k, dda.ALPHA_CM_RR, kh, e)
        P = np.linalg.solve(T, e)
        aj = 1.0 / dda.inverse_polarizability(M3[j], k, dda.ALPHA_CM_RR)
        assert np.allclose(P, aj * e, atol=1e-14)
    for e in (np.array([1.0, 0.0, 0.0]), np.array([0.3, 0.8, 0.0]) / np.hypot(0.3, 0.8),
              np.array([1.0, 1j, 0.0]) / np.sqrt(2)):
        T = dda.anisotropic_inverse_polarizability(M3, ang, k, dda.ALPHA_CM_RR, kh, e)
        E = e[None, :].astype(np.complex128)
        P = dda.solve_dense(r, k, T[None], E)
        qext, qabs, qsca = dda.cross_sections(k, E, P, T[None])
        csca_closed = (8 * np.pi / 3) * k ** 4 * np.sum(np.abs(P) ** 2) / (np.pi * dda.effective_radius(1) ** 2)
        assert abs(qsca - csca_closed) <= 1e-12 * abs(csca_closed)
        # the scalar sum with the mean of the diagonal misses it (the tensor form matters)
        qabs_scalar = dda.cross_sections(k, E, P, np.array([np.trace(T) / 3]))[1]
        assert abs(qabs_scalar - qabs) > 1e-6 * abs(qabs)


def _cube():
    occ = np.ones((2, 3, 3), np.uint8)  # 3 x 3 x 2 sites, symmetric under 90 degrees about z
    return dda.sites_from_occupancy(occ)


def test_matrix_with_tensor_sites_is_symmetric():
    r, comp, _ = _cube()
    T = dda.anisotropic_inverse_polarizability(M3, (0.3, 0.5, 0.7), 0.4, dda.ALPHA_LDR, [0, 0, 1.0], [1.0, 0, 0])
    A = dda.dense_matrix(r, 0.4, np.repeat(T[None], len(r), axis=0))
    assert np.allclose(A, A.T, atol=1e-13 * np.abs(A).max())


def test_rotation_covariance():
    """Material axis along x, wave along z polarized along y, against the
    same with everything rotated by 90 degrees about z (axis along y,
    polarization along -x): P_B(R r_j) = R P_A(r_j)."""
    r, comp, _ = _cube()
    k = 0.5
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    kh = np.array([0.0, 0.0, 1.0])
    eA = np.array([0.0, 1.0, 0.0])
    eB = R @ eA
    TA = dda.anisotropic_inverse_polarizability(M3, (0.0, 0.0, 0.0), k, dda.ALPHA_LDR, kh, eA)
    TB = dda.anisotropic_inverse_polarizability(M3, (np.pi / 2, 0.0, 0.0), k, dda.ALPHA_LDR, kh, eB)
    assert np.allclose(dda.dielectric_frame(np.pi / 2, 0, 0)[0], R @ [1, 0, 0])
    n = len(r)
    PA = dda.solve_dense(r, k, np.repeat(TA[None], n, axis=0), dda.incident_field(r, k, kh, eA))
    PB = dda.solve_dense(r, k, np.repeat(TB[None], n, axis=0), dda.incident_field(r, k, kh, eB))
    rot = r @ R.T
    for j in range(n):
        i = int(np.argmin(np.sum((r - rot[j]) ** 2, axis=1)))
        assert np.allclose(r[i], rot[j])
        assert np.allclose(PB[i], R @ PA[j], atol=1e-12 * np.abs(PA).max())
    # and the anisotropy matters: the isotropic solve differs
    Piso = dda.solve_dense(r, k, np.full(n, dda.inverse_polarizability(M3[1], k, dda.ALPHA_LDR, kh, eA)),
                           dda.incident_field(r, k, kh, eA))
    assert np.linalg.norm(Piso - PA) > 1e-3 * np.linalg.norm(PA)
