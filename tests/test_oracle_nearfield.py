"""Pins of the near-field oracle (oracle/nearfield.py): the DDA's own
equation (the field at a dipole from the incident wave and all other dipoles
is the local field 1/alpha P, section "Choice of Iterative Algorithm", eq.
AP=E), Faraday's law curl E = i k B for the dipole fields, the incident wave's
B, and the far-field limit of the scattered field (the scattering amplitude)."""
import numpy as np
import pytest

import synth
from oracle import dda, nearfield


def _solved(kind=dda.ALPHA_LDR):
    occ = synth.ellipsoid_occupancy((6, 5, 5), (5.8, 4.6, 4.4))
    r, comp, _ = dda.sites_from_occupancy(occ)
    k, m = 0.5, 1.6 + 0.2j
    kh, es, _ = dda.waves_for_orientation(0.4, 1.0, 0.3)
    ainv = dda.site_inverse_polarizability(comp, [m], k, kind, kh, es[0])
    E = dda.incident_field(r, k, kh, es[0])
    P = dda.solve_dense(r, k, ainv, E)
    return r, k, kh, es[0], ainv, P


def test_field_at_each_dipole_is_its_local_field():
    r, k, kh, e0, ainv, P = _solved()
    E, B = nearfield.near_field(r, P, k, kh, e0, r)
    want = ainv[:, None] * P
    assert np.linalg.norm(E - want) / np.linalg.norm(want) < 1e-11


@pytest.mark.parametrize("seed", range(3))
def test_dipole_fields_obey_faraday(seed):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    k = 0.3 + rng.random()
    x = rng.standard_normal(3) * 2.0 + np.array([0.0, 0.0, 3.0])
    h = 1e-4
    E = lambda y: nearfield.dipole_fields(np.asarray(y)[None, :], p, k)[0][0]
    d = [(E(x + h * np.eye(3)[a]) - E(x - h * np.eye(3)[a])) / (2 * h) for a in range(3)]  # d[a][b] = dE_b / dx_a
    curl = np.array([d[1][2] - d[2][1], d[2][0] - d[0][2], d[0][1] - d[1][0]])
    B = nearfield.dipole_fields(x[None, :], p, k)[1][0]
    assert np.allclose(curl, 1j * k * B, rtol=1e-6, atol=1e-9 * np.abs(B).max())


def test_incident_wave_magnetic_field():
    r, k, kh, e0, ainv, P = _solved()
    pts = np.array([[40.0, -25.0, 33.0]])
    E, B = nearfield.near_field(r, np.zeros_like(P), k, kh, e0, pts)
    assert np.allclose(B[0], np.cross(kh, E[0]), atol=1e-14)
    assert np.allclose(E[0], e0 * np.exp(1j * k * pts[0] @ kh), atol=1e-14)


def test_far_field_is_the_scattering_amplitude():
    r, k, kh, e0, ainv, P = _solved()
    n = np.array([0.3, -0.5, 0.81])
    n /= np.linalg.norm(n)
    dist = 1e7
    E, B = nearfield.near_field(r, P, k, kh, np.zeros(3), (dist * n)[None, :])
    F = (P * np.exp(-1j * k * (r @ n))[:, None]).sum(0)
    want = k * k * np.exp(1j * k * dist) / dist * (F - n * (n @ F))
    assert np.linalg.norm(E[0] - want) / np.linalg.norm(want) < 1e-5
    assert np.linalg.norm(B[0] - np.cross(n, E[0])) / np.linalg.norm(want) < 1e-5
