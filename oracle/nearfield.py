"""E and B in or near the target from the dipole polarizations (test
infrastructure only).

The guide's section "Postprocessing: Calculating E and B In or Near the
Target" describes the total field at a point as the incident plane wave plus
the fields of all the oscillating point dipoles, with retardation. For a
dipole p at separation R = R n̂, wavenumber k, Gaussian units and time
dependence exp(-i omega t), the fields are the textbook ones:

    E = exp(i k R) [ k^2 / R (p - n̂ (n̂ . p)) + (1 / R^3 - i k / R^2) (3 n̂ (n̂ . p) - p) ]
      = -A(R) p   (A: the interaction block of ``dda.interaction_block``)
    B = k^2 exp(i k R) (1 / R + i / (k R^2)) (n̂ x p)

The incident wave contributes E_inc = e0 exp(i k khat . r) and
B_inc = khat x E_inc. A point that coincides with a dipole takes no
contribution from that dipole, which leaves the local field the dipole
responds to.

Reading: for points within d of a dipole the guide multiplies each
contribution by a smoothing factor phi(r) taken from a paper it cites but
does not print (Draine & Flatau 2008). This oracle, like the GPU library,
evaluates the bare dipole sum everywhere: parity unpinned for what the guide
would print within d of a dipole.
"""
from __future__ import annotations

import numpy as np


def dipole_fields(R, p, k):
    """(E, B) at separations R (M, 3) from a dipole p (3,) complex."""
    R = np.asarray(R, dtype=np.float64)
    r = np.sqrt((R * R).sum(-1))
    n = R / r[:, None]
    ph = np.exp(1j * k * r)
    np_ = n @ p
    far = (k * k / r)[:, None] * (p[None, :] - n * np_[:, None])
    near = (1.0 / r ** 3 - 1j * k / r ** 2)[:, None] * (3.0 * n * np_[:, None] - p[None, :])
    E = ph[:, None] * (far + near)
    B = (k * k * ph * (1.0 / r + 1j / (k * r * r)))[:, None] * np.cross(n, p[None, :])
    return E, B


def near_field(r_sites, P, k, khat, e0, points):
    """Total E and B (npts, 3) complex at `points` (TF, lattice units, same
    origin as the sites) for one incident wave (khat, e0) and its solution P
    (N, 3)."""
    points = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    r_sites = np.asarray(r_sites, dtype=np.float64)
    P = np.asarray(P, dtype=np.complex128)
    khat = np.asarray(khat, dtype=np.float64)
    e0 = np.asarray(e0, dtype=np.complex128)
    Einc = e0[None, :] * np.exp(1j * k * (points @ khat))[:, None]
    E = Einc.copy()
    B = np.cross(khat[None, :], Einc)
    for i, x in enumerate(points):
        R = x[None, :] - r_sites
        keep = (R * R).sum(-1) > 1e-18
        for j in np.nonzero(keep)[0]:
            e, b = dipole_fields(R[j:j + 1], P[j], k)
            E[i] += e[0]
            B[i] += b[0]
    return E, B
