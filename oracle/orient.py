"""Orientational sampling and averaging, and cross sections at other target
rotations Phi from two polarization solutions (test infrastructure only).

DDSCAT 7.1 guide:

* section "Sampling in Theta, Phi, and beta": beta and Phi take the midpoints
  of NBETA (NPHI) equal intervals of their ranges; Theta is sampled uniformly
  in cos(Theta): with odd NTHETA the values include both ends of the range
  (Simpson's rule in cos(Theta)), with even NTHETA they are the midpoints of
  NTHETA equal intervals of cos(Theta) (plain average);
* section "Orientational Averaging": each orientation is weighted by
  WGTA(Theta, Phi) x WGTB(beta), WGTB = 1/NBETA, WGTA = 1/(NTHETA NPHI) for
  even NTHETA and Simpson weights for odd NTHETA;
* section "Scattering by Finite Targets" (the IORTH remark): solutions for
  two orthogonal incident polarizations at one orientation give, by linear
  combination, the solution at any other Phi (a rotation of the target about
  the incidence direction), because the incidence direction in the target
  frame does not depend on Phi.  This is exact when the polarizability does
  not depend on the polarization (Clausius-Mossotti); the lattice-dispersion
  polarizability depends on it through S, so there it is an approximation.

Reading (the guide's printed Simpson weights): the guide gives WGTA =
(1/3 or 4/3 or 2/3)/(NTHETA x NPHI) for odd NTHETA, which does not sum to one
(NTHETA = 3 gives 2/3).  Simpson's rule over NTHETA - 1 intervals of
cos(Theta), divided by the length of the interval, gives (1, 4, 2, ..., 4, 1)
/ (3 (NTHETA - 1)); the oracle uses that normalized form, i.e. the printed
numerators over (NTHETA - 1) NPHI.  With NTHETA = 1 the single value is
THETMI with weight one.
"""
from __future__ import annotations

import numpy as np

from . import dda


def midpoints(lo: float, hi: float, n: int) -> np.ndarray:
    """Midpoints of n equal intervals of [lo, hi] (the beta and Phi rule)."""
    if n < 1:
        raise ValueError("need at least one sample")
    return lo + (np.arange(n) + 0.5) * (hi - lo) / n


def theta_samples(thetmi: float, thetmx: float, n: int) -> np.ndarray:
    """Theta values, uniform in cos(Theta) between cos(thetmi) and cos(thetmx):
    odd n includes both ends, even n takes interval midpoints (radians)."""
    if n < 1:
        raise ValueError("need at least one sample")
    c0, c1 = np.cos(thetmi), np.cos(thetmx)
    if n == 1:
        return np.array([thetmi], dtype=np.float64)
    if n % 2 == 1:
        u = c0 + np.arange(n) * (c1 - c0) / (n - 1)
    else:
        u = c0 + (np.arange(n) + 0.5) * (c1 - c0) / n
    return np.arccos(np.clip(u, -1.0, 1.0))


def theta_weights(n: int) -> np.ndarray:
    """Weights over the n Theta samples, summing to one: Simpson's rule in
    cos(Theta) for odd n >= 3, equal weights for even n, one for n = 1."""
    if n == 1:
        return np.ones(1)
    if n % 2 == 0:
        return np.full(n, 1.0 / n)
    w = np.ones(n)
    w[1:-1:2] = 4.0
    w[2:-1:2] = 2.0
    return w / (3.0 * (n - 1))


def orientation_samples(lims, counts):
    """beta, Theta, Phi samples and the weight of every (beta, Theta, Phi).

    lims: (BETAMI, BETAMX, THETMI, THETMX, PHIMIN, PHIMAX) in radians;
    counts: (NBETA, NTHETA, NPHI).  Returns (beta (nb,), theta (nt,),
    phi (np,), weight (nb, nt, np)) with weight = WGTB x WGTA.
    """
    nb, nt, nph = (int(v) for v in counts)
    beta = midpoints(lims[0], lims[1], nb)
    theta = theta_samples(lims[2], lims[3], nt)
    phi = midpoints(lims[4], lims[5], nph)
    w = (np.full(nb, 1.0 / nb)[:, None, None] * theta_weights(nt)[None, :, None]
         * np.full(nph, 1.0 / nph)[None, None, :])
    return beta, theta, phi, w


def orientational_average(values, weight):
    """sum over (beta, Theta, Phi) of weight x value; values (nb, nt, np, ...)."""
    v = np.asarray(values)
    return np.tensordot(weight, v, axes=([0, 1, 2], [0, 1, 2]))


def phi_coefficients(beta, theta, phi_ref, phi, e01_lab=(0, 1, 0)):
    """c[l, a] with e_l(beta, theta, phi) = sum_a c[l, a] e_a(beta, theta, phi_ref),
    target-frame polarization vectors of the two incident states.  Both
    orientations share the incidence direction, and the reference vectors are
    orthonormal (e_a^* . e_b = delta_ab), so c[l, a] = e_a^* . e_l."""
    kr, er, _ = dda.waves_for_orientation(beta, theta, phi_ref, e01_lab)
    k, e, _ = dda.waves_for_orientation(beta, theta, phi, e01_lab)
    if not np.allclose(kr, k, atol=1e-12):
        raise ValueError("orientations differ in more than Phi")
    return e @ np.conj(er).T


def combine_pair(c, X):
    """X_l = sum_a c[l, a] X_a for a pair X (2, ...) of fields or solutions."""
    return np.tensordot(np.asarray(c), np.asarray(X), axes=([1], [0]))


def cross_sections_at_phi(k, E_pair, P_pair, ainv, c, n_dipoles=None):
    """(Q_ext, Q_abs, Q_sca) for both incident states at the rotated
    orientation, from the reference pair's fields and solutions; ainv is the
    per-site 1/alpha (independent of the polarization)."""
    E = combine_pair(c, E_pair)
    P = combine_pair(c, P_pair)
    return [dda.cross_sections(k, E[l], P[l], ainv, n_dipoles) for l in range(2)]
