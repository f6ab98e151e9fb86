"""Pins for the oracle's frame conventions (guide, section "Target Orientation"
and "Incident Polarization State")."""
import os

import numpy as np
import pytest

from oracle import dda

GOLD = os.path.join(os.path.dirname(__file__), "golden", "orientation_cases.txt")


def _cases():
    out = []
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if not line:
            continue
        parts = [p.split() for p in line.split("|")]
        case, th, ph, be = parts[0][0], *map(float, parts[0][1:4])
        axes = np.array([list(map(float, p)) for p in parts[1:4]])
        out.append((int(case), th, ph, be, axes))
    return out


@pytest.mark.parametrize("case,theta,phi,beta,axes", _cases())
def test_printed_orientation_cases(case, theta, phi, beta, axes):
    """The guide's 14 worked orientation cases (a1 = x_TF, a2 = y_TF)."""
    L = dda.lab_axes_in_target_frame(np.deg2rad(beta), np.deg2rad(theta), np.deg2rad(phi))
    assert np.allclose(L, axes, atol=2e-6), (case, L)


def test_text_examples_target_axes():
    """Theta=90, Phi=0, beta=0 gives a1 = y_LF, a2 = -x_LF; beta=90 gives a2 = z_LF."""
    A = dda.target_axes_in_lab_frame(0.0, np.pi / 2, 0.0)
    assert np.allclose(A[0], [0, 1, 0]) and np.allclose(A[1], [-1, 0, 0])
    A = dda.target_axes_in_lab_frame(np.pi / 2, np.pi / 2, 0.0)
    assert np.allclose(A[0], [0, 1, 0]) and np.allclose(A[1], [0, 0, 1])


@pytest.mark.parametrize("seed", range(5))
def test_two_printed_rotations_are_inverse(seed):
    """The two printed sets of equations (target axes in the LF, LF axes over
    the target axes) describe the same rotation: one is the transpose of the
    other, and both are proper rotations."""
    rng = np.random.default_rng(seed)
    b, t, p = rng.uniform(-np.pi, np.pi, 3)
    L = dda.lab_axes_in_target_frame(b, t, p)
    A = dda.target_axes_in_lab_frame(b, t, p)
    assert np.allclose(L, A.T, atol=1e-14)
    assert np.allclose(L @ L.T, np.eye(3), atol=1e-14)
    assert np.isclose(np.linalg.det(L), 1.0)


def test_second_polarization_examples():
    """e01 = y gives e02 = z; e01 = (y + i z)/sqrt2 (given unnormalized as
    (0, 1, i)) gives e02 = (i y + z)/sqrt2."""
    e1, e2 = dda.incident_polarizations((0, 1, 0))
    assert np.allclose(e2, [0, 0, 1])
    e1, e2 = dda.incident_polarizations((0, 1, 1j))
    assert np.allclose(e1, np.array([0, 1, 1j]) / np.sqrt(2))
    assert np.allclose(e2, np.array([0, 1j, 1]) / np.sqrt(2))
    assert abs(np.vdot(e1, e2)) < 1e-15


def test_waves_in_target_frame():
    """khat is x_LF in the TF; the polarizations are transverse and unit."""
    for b, t, p in [(0.3, 1.1, 2.0), (1.0, 0.2, -0.7)]:
        khat, e, L = dda.waves_for_orientation(b, t, p, e01_lab=(0, 1, 1j))
        assert np.allclose(khat, L[0])
        for ev in e:
            assert abs(np.dot(khat, ev)) < 1e-14
            assert np.isclose(np.vdot(ev, ev).real, 1.0)
