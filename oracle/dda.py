"""CPU oracle for the discrete dipole approximation (test infrastructure only).

Plain, slow, double-precision reference for everything the GPU library
computes.  It shares no code with the GPU path: only ``tests/``, the smoke
check and the benchmark's CPU-baseline leg may import it.

The DDSCAT 7.1 guide states the system to solve (section "Choice of Iterative
Algorithm", eq. AP=E), the target description, orientation and polarization
conventions, and the scattering-amplitude and Mueller-matrix relations; it
cites but does not print the interaction tensor, the polarizabilities and the
cross-section sums.  For those the oracle writes out the standard definitions
from the cited literature (Draine 1988; Draine & Goodman 1993), and says so
at each function.

Units: lattice spacing d = 1, incident amplitude |E0| = 1, Gaussian units,
time dependence exp(-i omega t).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# Lattice-dispersion-relation coefficients of Draine & Goodman (1993), the
# reference the guide cites for the LATTDR polarizability (section "Dipole
# Polarizabilities").  The guide does not print them: parity unpinned.
LDR_B1 = -1.8915316
LDR_B2 = 0.1648469
LDR_B3 = -1.7700004

ALPHA_CM = "cm"        # Clausius-Mossotti, no radiative reaction
ALPHA_CM_RR = "cm_rr"  # Clausius-Mossotti with the radiative-reaction term
ALPHA_LDR = "ldr"      # lattice dispersion relation (LATTDR)


# ---------------------------------------------------------------------------
# Target: occupied lattice sites
# ---------------------------------------------------------------------------

def sites_from_occupancy(occ: np.ndarray, origin=None):
    """Occupied sites of an occupancy grid (shape (n3, n2, n1), x fastest).

    Returns (r, comp, idx): r (N, 3) float64 site coordinates relative to the
    target-frame origin, comp (N,) int composition ids (>= 1), idx (N, 3) int
    lattice indices (ix, iy, iz).  Sites are listed in increasing linear box
    index ix + n1 (iy + n2 iz).  The origin defaults to the centroid of the
    occupied sites (the guide's ELLIPSOID entry puts the target-frame origin
    at the centroid).
    """
    occ = np.asarray(occ)
    iz, iy, ix = np.nonzero(occ)  # C order => sorted by linear index
    idx = np.stack([ix, iy, iz], axis=1).astype(np.int64)
    comp = occ[iz, iy, ix].astype(np.int64)
    if origin is None:
        origin = idx.mean(axis=0) if len(idx) else np.zeros(3)
    r = idx.astype(np.float64) - np.asarray(origin, dtype=np.float64)[None, :]
    return r, comp, idx


def effective_radius(n_dipoles: int) -> float:
    """a_eff = (3 V / 4 pi)^(1/3) with V = N d^3 (section "Applicability of the DDA")."""
    return (3.0 * n_dipoles / (4.0 * np.pi)) ** (1.0 / 3.0)


# ---------------------------------------------------------------------------
# Frames (section "Target Orientation")
# ---------------------------------------------------------------------------

def lab_axes_in_target_frame(beta, theta, phi, a1=(1.0, 0.0, 0.0), a2=(0.0, 1.0, 0.0)):
    """Target-frame components of the lab axes x_LF, y_LF, z_LF.

    Follows the expansion of x_LF, y_LF, z_LF over the target axes a1, a2,
    a3 = a1 x a2 given in "Orientation of the Target in the Lab Frame".
    Angles in radians.  Returns a (3, 3) array whose rows are x_LF, y_LF, z_LF.
    """
    a1 = np.asarray(a1, dtype=np.float64)
    a2 = np.asarray(a2, dtype=np.float64)
    a1 = a1 / np.linalg.norm(a1)
    a2 = a2 / np.linalg.norm(a2)
    a3 = np.cross(a1, a2)
    cb, sb = np.cos(beta), np.sin(beta)
    ct, st = np.cos(theta), np.sin(theta)
    cp, sp = np.cos(phi), np.sin(phi)
    xl = a1 * ct - a2 * st * cb + a3 * st * sb
    yl = a1 * st * cp + a2 * (ct * cb * cp - sb * sp) - a3 * (ct * sb * cp + cb * sp)
    zl = a1 * st * sp + a2 * (ct * cb * sp + sb * cp) - a3 * (ct * sb * sp - cb * cp)
    return np.stack([xl, yl, zl])


def target_axes_in_lab_frame(beta, theta, phi):
    """Lab-frame components of a1, a2, a3 (same section, first set of equations)."""
    cb, sb = np.cos(beta), np.sin(beta)
    ct, st = np.cos(theta), np.sin(theta)
    cp, sp = np.cos(phi), np.sin(phi)
    a1 = np.array([ct, st * cp, st * sp])
    a2 = np.array([-st * cb, ct * cb * cp - sb * sp, ct * cb * sp + sb * cp])
    a3 = np.array([st * sb, -(ct * sb * cp + cb * sp), -(ct * sb * sp - cb * cp)])
    return np.stack([a1, a2, a3])


def incident_polarizations(e01_lab=(0, 1, 0)):
    """Normalized e01 and e02 = x_LF x conj(e01), lab-frame components.

    Section "Incident Polarization State": the user's e01 is normalized and
    the second state is built as x_LF cross e01*.
    """
    e01 = np.asarray(e01_lab, dtype=np.complex128)
    e01 = e01 / np.sqrt(np.vdot(e01, e01).real)
    xhat = np.array([1.0, 0.0, 0.0], dtype=np.complex128)
    e02 = np.cross(xhat, np.conj(e01))
    return e01, e02


def waves_for_orientation(beta, theta, phi, e01_lab=(0, 1, 0), a1=(1, 0, 0), a2=(0, 1, 0)):
    """Target-frame incidence direction and the two polarization vectors.

    Returns (khat_tf (3,), [e1_tf, e2_tf] complex (2, 3), lab_axes (3, 3)).
    """
    L = lab_axes_in_target_frame(beta, theta, phi, a1, a2)
    e01, e02 = incident_polarizations(e01_lab)
    khat = L[0].copy()
    e1 = e01[0] * L[0] + e01[1] * L[1] + e01[2] * L[2]
    e2 = e02[0] * L[0] + e02[1] * L[1] + e02[2] * L[2]
    return khat, np.stack([e1, e2]), L


# ---------------------------------------------------------------------------
# Incident field and polarizability
# ---------------------------------------------------------------------------

def incident_field(r, k, khat, e):
    """E_j = e exp(i k khat . r_j) at every site; (N, 3) complex."""
    ph = np.exp(1j * k * (r @ np.asarray(khat, dtype=np.float64)))
    return ph[:, None] * np.asarray(e, dtype=np.complex128)[None, :]


def clausius_mossotti(m):
    """alpha_CM = (3 / 4 pi) (eps - 1) / (eps + 2), eps = m^2, d = 1."""
    eps = np.asarray(m, dtype=np.complex128) ** 2
    return (3.0 / (4.0 * np.pi)) * (eps - 1.0) / (eps + 2.0)


def inverse_polarizability(m, k, kind=ALPHA_LDR, khat=None, e=None):
    """1/alpha for refractive index m (per composition) at wavenumber k (d = 1).

    CM:    1/alpha_CM.
    CM_RR: 1/alpha_CM - (2/3) i k^3 (radiative reaction).
    LDR:   1/alpha_CM + (b1 + eps b2 + eps b3 S) k^2 - (2/3) i k^3, with
           S = sum_j (khat_j e_j)^2 (Draine & Goodman 1993); for complex e the
           reading S = sum_j khat_j^2 |e_j|^2 is taken.
    """
    m = np.asarray(m, dtype=np.complex128)
    eps = m ** 2
    inv = 1.0 / clausius_mossotti(m)
    if kind == ALPHA_CM:
        return inv
    if kind == ALPHA_CM_RR:
        return inv - (2.0 / 3.0) * 1j * k ** 3
    if kind == ALPHA_LDR:
        kh = np.asarray(khat, dtype=np.float64)
        ev = np.asarray(e, dtype=np.complex128)
        S = float(np.sum(kh ** 2 * np.abs(ev) ** 2))
        return inv + (LDR_B1 + eps * LDR_B2 + eps * LDR_B3 * S) * k ** 2 - (2.0 / 3.0) * 1j * k ** 3
    raise ValueError(kind)


def dielectric_frame(theta_df, phi_df, beta_df):
    """Target-frame components of the principal axes e_1, e_2, e_3 of a
    dielectric tensor whose Dielectric Frame is rotated by (Theta_DF, Phi_DF,
    beta_DF) from the Target Frame ("Composite Targets with Anisotropic
    Constituents": rotate by Theta_DF about y_TF, by Phi_DF about x_TF, then
    by beta_DF about e_1; the guide's expansion of e_1, e_2, e_3).  Returns a
    (3, 3) array whose rows are e_1, e_2, e_3."""
    ct, st = np.cos(theta_df), np.sin(theta_df)
    cp, sp = np.cos(phi_df), np.sin(phi_df)
    cb, sb = np.cos(beta_df), np.sin(beta_df)
    e1 = np.array([ct, st * cp, st * sp])
    e2 = np.array([-st * cb, ct * cb * cp - sb * sp, ct * cb * sp + sb * cp])
    e3 = np.array([st * sb, -(ct * sb * cp + cb * sp), -(ct * sb * sp - cb * cp)])
    return np.stack([e1, e2, e3])


def anisotropic_inverse_polarizability(m3, angles, k, kind=ALPHA_LDR, khat=None, e=None):
    """Target-frame 3 x 3 tensor 1/alpha of a material with refractive index
    m3[j] along principal axis e_j of its Dielectric Frame (angles =
    (Theta_DF, Phi_DF, beta_DF), see dielectric_frame).  The polarizability
    is diagonal in the DF, each element from the prescription with eps_j =
    m3[j]^2 (for LDR with the incident k and polarization as for an
    isotropic site, S taken in the target frame of the lattice); in the TF
    alpha = sum_j alpha_j e_j e_j^T, so 1/alpha = sum_j (1/alpha_j) e_j e_j^T.
    Reading: the guide defines R_ij = x_i . e_j and writes alpha_TF = R
    alpha_DF R^-1 (a symmetric tensor), which is this sum; its printed matrix
    is the transpose of that definition."""
    ef = dielectric_frame(*angles)
    inv = [inverse_polarizability(mj, k, kind, khat, e) for mj in m3]
    return sum(inv[j] * np.outer(ef[j], ef[j]) for j in range(3))


def site_inverse_polarizability(comp, m_list, k, kind=ALPHA_LDR, khat=None, e=None):
    """Per-site 1/alpha (N,) from composition ids (1-based) and m per composition."""
    table = np.array([inverse_polarizability(mm, k, kind, khat, e) for mm in m_list])
    return table[np.asarray(comp) - 1]


# ---------------------------------------------------------------------------
# Interaction matrix (dense) and its action
# ---------------------------------------------------------------------------

def interaction_block(rvec, k):
    """A(r) for one nonzero separation r = r_j - r_l (3-vector): the 3x3 block

        exp(i k r)/r [ k^2 (n n - I) + (i k r - 1)/r^2 (3 n n - I) ],

    i.e. minus the dipole field tensor (Draine 1988; the guide cites it in
    its introduction and in "Choice of Iterative Algorithm")."""
    rr = float(np.sqrt(np.dot(rvec, rvec)))
    n = np.asarray(rvec, dtype=np.float64) / rr
    nn = np.outer(n, n)
    I3 = np.eye(3)
    return np.exp(1j * k * rr) / rr * (k * k * (nn - I3) + (1j * k * rr - 1.0) / rr ** 2 * (3.0 * nn - I3))


def dense_matrix(r, k, ainv):
    """The 3N x 3N matrix A of eq. AP=E, site-major (row 3 j + a).  ainv is
    1/alpha per site, (N,), or the per-site 3 x 3 tensor, (N, 3, 3)."""
    r = np.asarray(r, dtype=np.float64)
    n = len(r)
    A = np.zeros((3 * n, 3 * n), dtype=np.complex128)
    d = r[:, None, :] - r[None, :, :]
    rr = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(rr, 1.0)
    nv = d / rr[..., None]
    ph = np.exp(1j * k * rr) / rr
    c1 = k * k
    c2 = (1j * k * rr - 1.0) / rr ** 2
    for a in range(3):
        for b in range(3):
            nn = nv[..., a] * nv[..., b]
            delta = 1.0 if a == b else 0.0
            blk = ph * (c1 * (nn - delta) + c2 * (3.0 * nn - delta))
            np.fill_diagonal(blk, 0.0)
            A[a::3, b::3] = blk
    idx = np.arange(n)
    ainv = np.asarray(ainv)
    if ainv.ndim == 3:  # per-site 3 x 3 blocks (anisotropic sites)
        for a in range(3):
            for b in range(3):
                A[3 * idx + a, 3 * idx + b] = ainv[:, a, b]
    else:
        for a in range(3):
            A[3 * idx + a, 3 * idx + a] = ainv
    return A


def solve_dense(r, k, ainv, E):
    """P from LAPACK's LU solve of the dense system; E, P are (N, 3)."""
    A = dense_matrix(r, k, ainv)
    P = np.linalg.solve(A, np.asarray(E, dtype=np.complex128).reshape(-1))
    return P.reshape(-1, 3)


_LIB = None


def _direct_lib():
    global _LIB
    if _LIB is None:
        from . import build as _b

        path = _b.LIB
        if not os.path.exists(path):
            _b.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.oracle_matvec.argtypes = [ctypes.c_int64, P, ctypes.c_double, P, P, P]
        lib.oracle_matvec.restype = None
        lib.oracle_matvec_rows.argtypes = [ctypes.c_int64, P, ctypes.c_double, P, P,
                                           ctypes.c_int64, P, P]
        lib.oracle_matvec_rows.restype = None
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def matvec_direct(r, k, ainv, x):
    """y = A x by the direct O(N^2) pair sum (C + OpenMP); x, y are (N, 3)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    ainv = np.ascontiguousarray(np.broadcast_to(ainv, (len(r),)), dtype=np.complex128)
    x = np.ascontiguousarray(x, dtype=np.complex128).reshape(len(r), 3)
    y = np.empty_like(x)
    _direct_lib().oracle_matvec(len(r), r.ctypes.data, float(k), ainv.ctypes.data,
                                x.ctypes.data, y.ctypes.data)
    return y


def threads() -> int:
    """OpenMP threads used by the direct matvec."""
    return int(_direct_lib().oracle_threads())


def matvec_rows(r, k, ainv, x, rows):
    """(A x) at the listed sites only: (len(rows), 3)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    ainv = np.ascontiguousarray(np.broadcast_to(ainv, (len(r),)), dtype=np.complex128)
    x = np.ascontiguousarray(x, dtype=np.complex128).reshape(len(r), 3)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    y = np.empty((len(rows), 3), dtype=np.complex128)
    _direct_lib().oracle_matvec_rows(len(r), r.ctypes.data, float(k), ainv.ctypes.data,
                                     x.ctypes.data, len(rows), rows.ctypes.data, y.ctypes.data)
    return y


# ---------------------------------------------------------------------------
# Iterative solve (the oracle's own BiCGstab, van der Vorst 1992)
# ---------------------------------------------------------------------------

def bicgstab(matvec, b, x0=None, tol=1e-10, max_iter=10000):
    """Unpreconditioned BiCGstab for a general complex system A x = b.

    Stops when ||b - A x|| / ||b|| <= tol (residual recomputed at the end).
    Returns (x, info) with info = {iters, matvecs, rel_resid}.
    """
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.complex128).reshape(-1).copy()
    nb = np.linalg.norm(b)
    if nb == 0:
        return x, {"iters": 0, "matvecs": 0, "rel_resid": 0.0}
    r = b - matvec(x)
    nmv = 1
    rhat = r.copy()
    rho_old = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    it = 0
    while np.linalg.norm(r) / nb > tol and it < max_iter:
        rho = np.vdot(rhat, r)
        if it == 0:
            p = r.copy()
        else:
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
        v = matvec(p)
        alpha = rho / np.vdot(rhat, v)
        s = r - alpha * v
        t = matvec(s)
        nmv += 2
        tt = np.vdot(t, t).real
        omega = np.vdot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
        it += 1
    r_true = b - matvec(x)
    nmv += 1
    return x, {"iters": it, "matvecs": nmv, "rel_resid": float(np.linalg.norm(r_true) / nb)}


def bicgstab_l(matvec, b, ell=2, x0=None, tol=1e-10, max_iter=10000, keep_residuals=False):
    """BiCGstab(ell) for a general complex system A x = b (Sleijpen & Fokkema
    1993): each cycle takes ell BiCG steps, keeping the residuals r_0..r_ell
    and directions u_0..u_ell = A^i applied to the cycle's first ones, then
    replaces the ell one-dimensional minimisations of BiCGstab by one
    minimisation of ||r_0 - sum_j gamma_j r_j|| over a polynomial of degree
    ell (modified Gram-Schmidt on r_1..r_ell).  ell = 1 is BiCGstab.  The
    guide's default solver PBCGS2 is this method with ell = 2 (the routine
    ZBCG2, after Fokkema's thesis and Sleijpen & van der Vorst; "Choice of
    Iterative Algorithm").

    Inner products (a, b) = a^H b.  Stops at the end of the first cycle with
    ||r_0|| / ||b|| <= tol (r_0 is the residual of the current x throughout)
    or with max_iter BiCG steps taken, and recomputes the true residual at
    the end.  Returns (x, info) with info = {iters (BiCG steps, 2 matvecs
    each), matvecs, rel_resid} and info["residuals"], the recursive residual
    norms at the start and after each cycle, if keep_residuals."""
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.complex128).reshape(-1).copy()
    nb = np.linalg.norm(b)
    if nb == 0:
        return x, {"iters": 0, "matvecs": 0, "rel_resid": 0.0}
    r = [b - matvec(x)] + [None] * ell
    u = [np.zeros_like(b)] + [None] * ell
    nmv = 1
    rt = r[0].copy()  # shadow residual
    rho0, alpha, omega = 1.0 + 0j, 0.0 + 0j, 1.0 + 0j
    hist = [np.linalg.norm(r[0]) / nb]
    it = 0
    done = hist[0] <= tol
    while not done:
        rho0 = -omega * rho0
        # BiCG part
        for j in range(ell):
            rho1 = np.vdot(rt, r[j])
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = matvec(u[j])
            gamma = np.vdot(rt, u[j + 1])
            alpha = rho0 / gamma
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            r[j + 1] = matvec(r[j])
            x = x + alpha * u[0]
            nmv += 2
            it += 1
        # MR part: modified Gram-Schmidt on r_1..r_ell, then the polynomial
        tau = np.zeros((ell + 1, ell + 1), dtype=np.complex128)
        sigma = np.zeros(ell + 1)
        gp = np.zeros(ell + 1, dtype=np.complex128)
        for j in range(1, ell + 1):
            for i in range(1, j):
                tau[i, j] = np.vdot(r[i], r[j]) / sigma[i]
                r[j] = r[j] - tau[i, j] * r[i]
            sigma[j] = np.vdot(r[j], r[j]).real
            gp[j] = np.vdot(r[j], r[0]) / sigma[j]
        g = np.zeros(ell + 1, dtype=np.complex128)
        g[ell] = gp[ell]
        omega = g[ell]
        for j in range(ell - 1, 0, -1):
            g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, ell + 1))
        gpp = np.zeros(ell + 1, dtype=np.complex128)
        for j in range(1, ell):
            gpp[j] = g[j + 1] + sum(tau[j, i] * g[i + 1] for i in range(j + 1, ell))
        x = x + g[1] * r[0]
        r[0] = r[0] - gp[ell] * r[ell]
        u[0] = u[0] - g[ell] * u[ell]
        for j in range(1, ell):
            u[0] = u[0] - g[j] * u[j]
            x = x + gpp[j] * r[j]
            r[0] = r[0] - gp[j] * r[j]
        hist.append(np.linalg.norm(r[0]) / nb)
        done = hist[-1] <= tol or it >= max_iter
    r_true = b - matvec(x)
    nmv += 1
    info = {"iters": it, "matvecs": nmv, "rel_resid": float(np.linalg.norm(r_true) / nb)}
    if keep_residuals:
        info["residuals"] = hist
    return x, info


def cocg(matvec, b, x0=None, tol=1e-10, max_iter=10000, keep_residuals=False):
    """Conjugate orthogonal conjugate gradients for a complex symmetric
    A = A^T (the DDA matrix is one: A_jl = A_lj^T, and its diagonal is
    symmetric): CG with the bilinear form x^T y in place of x^H y (van der
    Vorst & Melissen 1990; the guide lists the complex-symmetric QMR family
    among the PIM methods, "Choice of Iterative Algorithm").  One matvec per
    iteration.  Stops when ||b - A x|| / ||b|| <= tol (residual recomputed at
    the end).  Returns (x, info) with info = {iters, matvecs, rel_resid}, and
    info["residuals"] (the recursive residuals) if keep_residuals."""
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.complex128).reshape(-1).copy()
    nb = np.linalg.norm(b)
    if nb == 0:
        return x, {"iters": 0, "matvecs": 0, "rel_resid": 0.0}
    r = b - matvec(x)
    nmv = 1
    p = r.copy()
    rho = r @ r
    res = [r.copy()] if keep_residuals else None
    it = 0
    while np.linalg.norm(r) / nb > tol and it < max_iter:
        q = matvec(p)
        nmv += 1
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rho_new = r @ r
        p = r + (rho_new / rho) * p
        rho = rho_new
        it += 1
        if keep_residuals:
            res.append(r.copy())
    r_true = b - matvec(x)
    nmv += 1
    info = {"iters": it, "matvecs": nmv, "rel_resid": float(np.linalg.norm(r_true) / nb)}
    if keep_residuals:
        info["residuals"] = res
    return x, info


def solve_iterative(r, k, ainv, E, tol=1e-10, x0=None, max_iter=10000):
    """P from BiCGstab over the direct matvec; E, P are (N, 3)."""
    n = len(r)
    mv = lambda v: matvec_direct(r, k, ainv, v.reshape(n, 3)).reshape(-1)
    x, info = bicgstab(mv, np.asarray(E).reshape(-1), None if x0 is None else np.asarray(x0).reshape(-1),
                       tol=tol, max_iter=max_iter)
    return x.reshape(n, 3), info


def residual_norms(r, k, ainv, E, P):
    """(||E - A P|| / ||E||, the guide's eq. err_tol value ||A^H A P - A^H E|| / ||A^H E||).

    A^H v is evaluated as conj(A conj(v)), valid because A is symmetric.
    """
    E = np.asarray(E, dtype=np.complex128)
    AP = matvec_direct(r, k, ainv, P)
    rvec = E - AP
    rel = np.linalg.norm(rvec) / np.linalg.norm(E)
    AH = lambda v: np.conj(matvec_direct(r, k, ainv, np.conj(v)))
    num = AH(rvec)
    den = AH(E)
    return float(rel), float(np.linalg.norm(num) / np.linalg.norm(den))


# ---------------------------------------------------------------------------
# Cross sections (Draine 1988 sums; Q = C / (pi a_eff^2), section
# "What Does It Calculate?")
# ---------------------------------------------------------------------------

def cross_sections(k, E, P, ainv, n_dipoles=None):
    """(Q_ext, Q_abs, Q_sca) with Q_sca = Q_ext - Q_abs.

    C_ext = 4 pi k sum_j Im(E_j^* . P_j)
    C_abs = 4 pi k sum_j [ Im(P_j . conj(1/alpha_j) P_j^*) - (2/3) k^3 |P_j|^2 ]

    ainv: 1/alpha per site (N,), or per-site 3 x 3 tensors (N, 3, 3), for
    which P_j . conj(1/alpha_j) P_j^* is the quadratic form.
    """
    E = np.asarray(E, dtype=np.complex128)
    P = np.asarray(P, dtype=np.complex128)
    n = len(P) if n_dipoles is None else n_dipoles
    cext = 4.0 * np.pi * k * np.sum(np.imag(np.conj(E) * P))
    p2 = np.sum(np.abs(P) ** 2, axis=1)
    ainv = np.asarray(ainv)
    if ainv.ndim == 3:
        # tensor 1/alpha: Im(P . (1/alpha)^* P^*) = Im(P^T conj(T) conj(P))
        quad = np.einsum("ja,jab,jb->j", P, np.conj(ainv), np.conj(P))
        cabs = 4.0 * np.pi * k * np.sum(np.imag(quad) - (2.0 / 3.0) * k ** 3 * p2)
    else:
        cabs = 4.0 * np.pi * k * np.sum(np.imag(np.conj(ainv)) * p2 - (2.0 / 3.0) * k ** 3 * p2)
    area = np.pi * effective_radius(n) ** 2
    qext, qabs = cext / area, cabs / area
    return float(qext), float(qabs), float(qext - qabs)


def scattering_double_sum(r, k, P):
    """C_sca / (pi a_eff^2) from the exact double sum over site pairs,

        C_sca = 4 pi k sum_j sum_l P_j^H Im[G(r_j - r_l)] P_l,

    with G = -A off the diagonal and Im G(0) = (2/3) k^3 I.  Equals
    k^4 times the integral of |sum_j (P_j - n (n . P_j)) exp(-i k n . r_j)|^2
    over directions; an identity only for a solution of A P = E when
    compared with Q_ext - Q_abs (optical theorem)."""
    r = np.asarray(r, dtype=np.float64)
    P = np.asarray(P, dtype=np.complex128)
    n = len(r)
    total = (2.0 / 3.0) * k ** 3 * np.sum(np.abs(P) ** 2)
    for j in range(n):
        d = r[j][None, :] - r
        rr = np.sqrt((d ** 2).sum(-1))
        mask = np.arange(n) != j
        d, rr, Pl = d[mask], rr[mask], P[mask]
        nv = d / rr[:, None]
        ph = np.exp(1j * k * rr) / rr
        nP = np.sum(nv * Pl, axis=1)
        # G P_l = -(A P_l) = ph [ k^2 (P - n (n.P)) + (1 - ikr)/r^2 (3 n (n.P) - P) ]
        GP = ph[:, None] * (k * k * (Pl - nv * nP[:, None])
                            + ((1.0 - 1j * k * rr) / rr ** 2)[:, None] * (3.0 * nv * nP[:, None] - Pl))
        # P_j^H Im[G] P_l with Im taken elementwise: Im G is real symmetric, so
        # sum_l P_j^H ImG P_l = Re over the pair sum of conj(P_j) . ImG P_l after
        # symmetrisation; compute Im G P_l as (G P_l - conj(G) P_l)/(2 i).
        GcP = np.conj(ph)[:, None] * (k * k * (Pl - nv * nP[:, None])
                                      + ((1.0 + 1j * k * rr) / rr ** 2)[:, None] * (3.0 * nv * nP[:, None] - Pl))
        ImGP = (GP - GcP) / 2j
        total += np.real(np.sum(np.conj(P[j])[None, :] * ImGP))
    csca = 4.0 * np.pi * k * total
    return float(csca / (np.pi * effective_radius(n) ** 2))


def shifted_previous_guess(r, k, P_prev, ainv_prev, ainv_new, khat_prev, khat_new):
    """Initial guess for the next wave of a sweep from the previous solution.

    The guide's default guess is P = 0 ("Choice of Iterative Algorithm"); a
    sweep over orientations may start instead from the previous orientation's
    polarization.  Its local field E_loc,j = (1/alpha_prev,j) P_prev,j is
    carried to the new incidence direction by the ratio of the two incident
    phases at the site, E_sh,j = E_loc,j exp(i k (khat_new - khat_prev) . r_j),
    and the guess is P0,j = E_sh,j / (1/alpha_new,j).  Returns (E_sh, P0), both
    (N, 3) complex; ainv_* are per-site (N,) arrays.
    """
    dk = k * (np.asarray(khat_new, dtype=float) - np.asarray(khat_prev, dtype=float))
    phase = np.exp(1j * (r @ dk))
    e_sh = (ainv_prev[:, None] * P_prev) * phase[:, None]
    return e_sh, e_sh / ainv_new[:, None]


def projected_history_guess(r, k, ainv_new, khat_new, E_new, history):
    """Least-squares initial guess over earlier solutions of a sweep.

    Each earlier solution (P, ainv, khat) in ``history`` is carried to the new
    incidence direction as in ``shifted_previous_guess``, giving v_e; the guess
    is P0 = sum_e c_e v_e with c minimising ||E_new - A P0||_2, the linear
    least-squares problem min_c ||E - W c|| with W = [A v_1 ... A v_h] (A of
    eq. AP=E with the new 1/alpha, by the direct matvec).  Returns (P0, c).
    """
    basis = [shifted_previous_guess(r, k, P, a, ainv_new, kh, khat_new)[1] for P, a, kh in history]
    W = np.stack([matvec_direct(r, k, ainv_new, v).reshape(-1) for v in basis], axis=1)
    c, *_ = np.linalg.lstsq(W, np.asarray(E_new).reshape(-1), rcond=None)
    return sum(ce * v for ce, v in zip(c, basis)), c
