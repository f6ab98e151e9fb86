"""Seeded synthetic inputs for the DDA solver and for its CPU oracle.

This module only *generates inputs*: occupancy grids of lattice targets,
refractive indices, size parameters and orientation angles.  It holds none
of the method's arithmetic (no polarizabilities, no interaction tensor, no
solver, no cross sections), so that both the GPU path and the oracle can be
fed the same seeded data without sharing any code that computes results.

Target shapes follow the ELLIPSOID target definition of the DDSCAT 7.1
guide (section "Target Generation: Isolated Finite Targets", ELLIPSOID
entry): a lattice site with target-frame coordinates (x, y, z) is occupied
when (x/D1)^2 + (y/D2)^2 + (z/D3)^2 <= 1/4, with D_i the diameters in units
of the lattice spacing.  Sites sit at half-integer offsets from the box
centre, so a sphere of diameter D = n fills an n^3 box symmetrically.

Occupancy arrays are uint8 with shape (n3, n2, n1) in C order, i.e. x is the
fastest index; value 0 is vacuum and c >= 1 names composition c.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "ellipsoid_occupancy",
    "sphere_occupancy",
    "random_ellipsoid",
    "aggregate_occupancy",
    "uniform_orientations",
    "theta_sweep",
    "mixed_box_targets",
    "CONFIG_SEED_BASE",
]

# Seeds are fixed per workload: CONFIG_SEED_BASE + workload number.
CONFIG_SEED_BASE = 1002150


def _centred_coords(n1: int, n2: int, n3: int):
    """Site coordinates relative to the box centre, at half-integer offsets."""
    x = np.arange(n1) + 0.5 - n1 / 2.0
    y = np.arange(n2) + 0.5 - n2 / 2.0
    z = np.arange(n3) + 0.5 - n3 / 2.0
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def ellipsoid_occupancy(dims, diam, rot=None, comp: int = 1) -> np.ndarray:
    """Occupancy of an ellipsoid with diameters ``diam`` (lattice units) in a box ``dims``.

    dims = (n1, n2, n3) with n1 along x.  ``rot`` is an optional 3x3 rotation
    whose columns are the ellipsoid's principal axes in the box frame.
    Returns uint8 array of shape (n3, n2, n1).
    """
    n1, n2, n3 = (int(d) for d in dims)
    X, Y, Z = _centred_coords(n1, n2, n3)
    if rot is not None:
        R = np.asarray(rot, dtype=np.float64)
        # coordinates along the principal axes
        U = R[0, 0] * X + R[1, 0] * Y + R[2, 0] * Z
        V = R[0, 1] * X + R[1, 1] * Y + R[2, 1] * Z
        W = R[0, 2] * X + R[1, 2] * Y + R[2, 2] * Z
        X, Y, Z = U, V, W
    d1, d2, d3 = (float(d) for d in diam)
    inside = (X / d1) ** 2 + (Y / d2) ** 2 + (Z / d3) ** 2 <= 0.25
    return (inside.astype(np.uint8) * np.uint8(comp))


def sphere_occupancy(n: int, diameter: float | None = None) -> np.ndarray:
    """Sphere of the given diameter (default n) centred in an n^3 box."""
    D = float(n if diameter is None else diameter)
    return ellipsoid_occupancy((n, n, n), (D, D, D))


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation (QR of a Gaussian matrix with sign fix)."""
    A = rng.standard_normal((3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def random_ellipsoid(n: int, rng: np.random.Generator):
    """Random-axis ellipsoid in an n^3 box.

    Axis ratios 1 : U[1,2] : U[1,3]; the principal axes are rotated at
    random, then the whole ellipsoid is scaled so that its bounding box just
    fits the n^3 box.  Returns (occupancy, diameters, rotation).
    """
    ratios = np.array([1.0, rng.uniform(1.0, 2.0), rng.uniform(1.0, 3.0)])
    R = _random_rotation(rng)
    # half-extent of the rotated ellipsoid along each box axis, per unit scale
    half = 0.5 * np.sqrt(((R * ratios[None, :]) ** 2).sum(axis=1))
    scale = (n / 2.0) / half.max()
    diam = ratios * scale
    occ = ellipsoid_occupancy((n, n, n), diam, rot=R)
    return occ, diam, R


def aggregate_occupancy(n: int, rng: np.random.Generator, corr_len: float = 4.0,
                        fill: float = 0.3, largest_component: bool = True) -> np.ndarray:
    """Porous aggregate: a thresholded, Gaussian-smoothed white-noise field.

    White noise on the n^3 box is smoothed with the kernel exp(-r^2/(2 l^2))
    (l = corr_len lattice units, periodic convolution) and thresholded at the
    (1 - fill) quantile.  Optionally only the largest 6-connected component is
    kept.  Returns uint8 occupancy (n, n, n).
    """
    noise = rng.standard_normal((n, n, n))
    f = np.fft.fftfreq(n)
    KZ, KY, KX = np.meshgrid(f, f, f, indexing="ij")
    k2 = (2 * np.pi) ** 2 * (KX ** 2 + KY ** 2 + KZ ** 2)
    field = np.fft.ifftn(np.fft.fftn(noise) * np.exp(-0.5 * corr_len ** 2 * k2)).real
    thr = np.quantile(field, 1.0 - fill)
    occ = field > thr
    if largest_component:
        from scipy import ndimage

        lab, nlab = ndimage.label(occ)
        if nlab > 1:
            sizes = np.bincount(lab.ravel())
            sizes[0] = 0
            occ = lab == int(np.argmax(sizes))
    return occ.astype(np.uint8)


def uniform_orientations(count: int, rng: np.random.Generator):
    """(beta, Theta, Phi) in radians, uniform over rotations: beta, Phi
    uniform in [0, 2 pi), cos(Theta) uniform in [-1, 1]."""
    beta = rng.uniform(0.0, 2 * np.pi, count)
    theta = np.arccos(rng.uniform(-1.0, 1.0, count))
    phi = rng.uniform(0.0, 2 * np.pi, count)
    return np.stack([beta, theta, phi], axis=1)


def theta_sweep(count: int, beta: float = 0.0, phi: float = 0.0):
    """A sweep of ``count`` consecutive orientations, uniform in cos(Theta)
    over [-1, 1] (interval midpoints), at fixed beta and Phi."""
    c = 1.0 - (np.arange(count) + 0.5) * (2.0 / count)
    th = np.arccos(c)
    return np.stack([np.full(count, beta), th, np.full(count, phi)], axis=1)



def mixed_box_targets(boxes, rng: np.random.Generator):
    """Targets of a mixed-box batch, one per box side in ``boxes``: a random
    ellipsoid (``random_ellipsoid``), a refractive index with Re m uniform in
    [1.2, 1.8] and Im m log-uniform in [0.001, 0.3], and a lattice wavenumber
    k d with |m| k d uniform in [0.3, 0.8].  Returns a list of
    (occupancy, m, kd), drawn in that order per target."""
    out = []
    for n in boxes:
        occ = random_ellipsoid(int(n), rng)[0]
        m = complex(rng.uniform(1.2, 1.8), np.exp(rng.uniform(np.log(1e-3), np.log(0.3))))
        kd = rng.uniform(0.3, 0.8) / abs(m)
        out.append((occ, m, kd))
    return out
