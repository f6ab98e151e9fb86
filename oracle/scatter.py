"""Oracle: scattering amplitudes, amplitude matrix S_1..S_4, Mueller matrix,
and angular-averaging quadrature (test infrastructure only).

Section "Scattering by Finite Targets: The Mueller Matrix" of the DDSCAT 7.1
guide defines f_ml through the scattered field (eq. f_ml_def), relates it to
the Bohren & Huffman amplitude matrix (eqs. S_ampl_def to
S_1_relto_f21andf22), and lists the 16 Mueller elements as bilinears in
S_1..S_4.  Section "Scattering Directions" fixes the lab-frame direction
n = x cos(theta) + y sin(theta) cos(phi) + z sin(theta) sin(phi).  Section
"Averaging over Scattering Directions" gives the solid-angle weights
(eq. average and the Omega_jk that follow) and the choice of scattering
angles from the parameter eta.
"""
from __future__ import annotations

import numpy as np


def lab_direction_basis(theta, phi):
    """Lab-frame n, theta_hat, phi_hat for scattering angles (theta, phi).

    theta_hat = dn/dtheta and phi_hat = (dn/dphi)/sin(theta), the spherical
    unit vectors about x_LF with phi measured from y_LF; at theta = 0 they
    reduce to e_i_par = y cos(phi) + z sin(phi) and -e_i_perp of eq.
    yz_vs_eis.  Returns three (..., 3) arrays.
    """
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    ct, st, cp, sp = np.cos(theta), np.sin(theta), np.cos(phi), np.sin(phi)
    n = np.stack([ct, st * cp, st * sp], axis=-1)
    th = np.stack([-st, ct * cp, ct * sp], axis=-1)
    ph = np.stack([np.zeros_like(cp), -sp, cp], axis=-1)
    return n, th, ph


def scattering_amplitudes(r, k, P_list, theta, phi, lab_axes):
    """f_ml(theta, phi) = k^3 e_m . sum_j P_j^(l) exp(-i k n . r_j).

    r: (N, 3) target-frame sites; P_list: list of (N, 3) solutions, one per
    incident polarization l; lab_axes: rows x_LF, y_LF, z_LF in the target
    frame.  e_1 = theta_hat, e_2 = phi_hat.  Returns f (ndir, 2, nl) complex.
    """
    n_lab, th_lab, ph_lab = lab_direction_basis(theta, phi)
    L = np.asarray(lab_axes, dtype=np.float64)
    n_tf, th_tf, ph_tf = n_lab @ L, th_lab @ L, ph_lab @ L
    phase = np.exp(-1j * k * (n_tf @ np.asarray(r, dtype=np.float64).T))  # (ndir, N)
    out = np.zeros((len(n_tf), 2, len(P_list)), dtype=np.complex128)
    for l, P in enumerate(P_list):
        F = phase @ np.asarray(P, dtype=np.complex128)  # (ndir, 3) = sum_j P_j e^{-ik n.r_j}
        out[:, 0, l] = k ** 3 * np.sum(th_tf * F, axis=1)
        out[:, 1, l] = k ** 3 * np.sum(ph_tf * F, axis=1)
    return out


def amplitude_matrix(f, phi, e01_lab, e02_lab):
    """S_1..S_4 from f_ml (guide eqs. following fml_rel_S_v4).

    a = e01* . y, b = e01* . z, c = e02* . y, d = e02* . z (lab frame).
    f: (ndir, 2, 2) with f[:, m-1, l-1].  Returns (ndir, 4) = (S1, S2, S3, S4).
    """
    e01 = np.asarray(e01_lab, dtype=np.complex128)
    e02 = np.asarray(e02_lab, dtype=np.complex128)
    a, b = np.conj(e01[1]), np.conj(e01[2])
    c, d = np.conj(e02[1]), np.conj(e02[2])
    cp, sp = np.cos(phi), np.sin(phi)
    f11, f12, f21, f22 = f[:, 0, 0], f[:, 0, 1], f[:, 1, 0], f[:, 1, 1]
    S1 = -1j * (f21 * (b * cp - a * sp) + f22 * (d * cp - c * sp))
    S2 = -1j * (f11 * (a * cp + b * sp) + f12 * (c * cp + d * sp))
    S3 = 1j * (f11 * (b * cp - a * sp) + f12 * (d * cp - c * sp))
    S4 = 1j * (f21 * (a * cp + b * sp) + f22 * (c * cp + d * sp))
    return np.stack([S1, S2, S3, S4], axis=-1)


def mueller(S):
    """The 4 x 4 Mueller matrix from S_1..S_4 (Bohren & Huffman bilinears as
    listed in "Relation Between Stokes Parameters of Incident and Scattered
    Radiation").  S: (..., 4).  Returns (..., 4, 4)."""
    S1, S2, S3, S4 = S[..., 0], S[..., 1], S[..., 2], S[..., 3]
    a1, a2, a3, a4 = (np.abs(S1) ** 2, np.abs(S2) ** 2, np.abs(S3) ** 2, np.abs(S4) ** 2)
    c = np.conj
    M = np.empty(S.shape[:-1] + (4, 4))
    M[..., 0, 0] = (a1 + a2 + a3 + a4) / 2
    M[..., 0, 1] = (a2 - a1 + a4 - a3) / 2
    M[..., 0, 2] = np.real(S2 * c(S3) + S1 * c(S4))
    M[..., 0, 3] = np.imag(S2 * c(S3) - S1 * c(S4))
    M[..., 1, 0] = (a2 - a1 + a3 - a4) / 2
    M[..., 1, 1] = (a1 + a2 - a3 - a4) / 2
    M[..., 1, 2] = np.real(S2 * c(S3) - S1 * c(S4))
    M[..., 1, 3] = np.imag(S2 * c(S3) + S1 * c(S4))
    M[..., 2, 0] = np.real(S2 * c(S4) + S1 * c(S3))
    M[..., 2, 1] = np.real(S2 * c(S4) - S1 * c(S3))
    M[..., 2, 2] = np.real(S1 * c(S2) + S3 * c(S4))
    M[..., 2, 3] = np.imag(S2 * c(S1) + S4 * c(S3))
    M[..., 3, 0] = np.imag(S4 * c(S2) + S1 * c(S3))
    M[..., 3, 1] = np.imag(S4 * c(S2) - S1 * c(S3))
    M[..., 3, 2] = np.imag(S1 * c(S2) - S3 * c(S4))
    M[..., 3, 3] = np.real(S1 * c(S2) - S3 * c(S4))
    return M


def linear_polarization(M):
    """P = (S21^2 + S31^2)^(1/2) / S11 for unpolarized incident light."""
    return np.sqrt(M[..., 1, 0] ** 2 + M[..., 2, 0] ** 2) / M[..., 0, 0]


def polarized_cross_sections(M, k, stokes_in):
    """dC_sca/dOmega of the scattered light that an ideal linear polarizer
    passes parallel (xi = 0) and perpendicular (xi = pi/2) to the scattering
    plane, and in total, per unit incident intensity (guide, "Polarization
    Properties of the Scattered Radiation": the polarizer's Mueller matrix
    applied to the scattered Stokes vector, which is M s_i / (k r)^2; and
    I_s r^2 = (dC_sca/dOmega) I_i, "Relation Between Mueller Matrix and
    Scattering Cross Sections").  M: (..., 4, 4); stokes_in: (I, Q, U, V)
    with I > 0.  Returns (..., 3): parallel, perpendicular, total."""
    s = np.asarray(stokes_in, dtype=np.float64)
    s = s / s[0]
    scat = np.einsum("...ij,j->...i", np.asarray(M, dtype=np.float64), s) / k ** 2  # r^2 I_s, Q_s, ... per I_i
    out = np.empty(scat.shape[:-1] + (3,))
    for n, xi in enumerate((0.0, np.pi / 2)):
        c2, s2 = np.cos(2 * xi), np.sin(2 * xi)
        out[..., n] = 0.5 * (scat[..., 0] + c2 * scat[..., 1] + s2 * scat[..., 2])
    out[..., 2] = scat[..., 0]
    return out


def scattering_theta_grid(x, eta):
    """theta_j (j = 1..N_theta) from the s(theta) = theta + theta/(theta+theta0)
    prescription with theta0 = 2 pi / (1 + x) ("Selection of Scattering
    Angles").  N_theta is rounded to the nearest integer >= 3 (reading: the
    guide gives a real-valued expression)."""
    th0 = 2 * np.pi / (1 + x)
    nth = 1 + 2 * (3 + x) / eta * (1 + 1 / (np.pi + th0)) / (1 + th0 / (np.pi + th0) ** 2)
    nth = max(3, int(np.rint(nth)))
    j = np.arange(1, nth + 1)
    s = (j - 1) * np.pi / (nth - 1) * (1 + 1 / (np.pi + th0))
    th = ((s - 1 - th0) + np.sqrt((1 + th0 - s) ** 2 + 4 * th0 * s)) / 2
    th[0], th[-1] = 0.0, np.pi
    return th


def scattering_directions(x, eta):
    """Directions (theta_j, phi_jk) and solid-angle weights Omega_jk.

    N_phi(j) = max{3, nint[4 pi sin(theta_j) / (theta_{j+1} - theta_{j-1})]}
    for interior j, one direction at theta = 0 and at theta = pi, and
    Omega_jk from the formulas under eq. average.  Returns (theta, phi, w)
    flat arrays; sum(w) is close to 4 pi.
    """
    th = scattering_theta_grid(x, eta)
    nth = len(th)
    T, Ph, W = [], [], []
    for j in range(nth):
        if j == 0 or j == nth - 1:
            nphi = 1
        else:
            nphi = max(3, int(np.rint(4 * np.pi * np.sin(th[j]) / (th[j + 1] - th[j - 1]))))
        if j == 0:
            w = 2 * np.pi / nphi * (1 - (np.cos(th[0]) + np.cos(th[1])) / 2)
        elif j == nth - 1:
            w = 2 * np.pi / nphi * ((np.cos(th[-2]) + np.cos(th[-1])) / 2 + 1)
        else:
            w = np.pi / nphi * (np.cos(th[j - 1]) - np.cos(th[j + 1]))
        for kk in range(nphi):
            T.append(th[j])
            Ph.append(2 * np.pi * kk / nphi)
            W.append(w)
    return np.array(T), np.array(Ph), np.array(W)


def scattering_quadrature(r, k, P, lab_axes, x, eta=0.5):
    """Q_sca from sum_jk Omega_jk k^4 |sum_j (P_j - n (n.P_j)) e^{-ik n.r_j}|^2 / (pi a_eff^2).

    A third, approximate route to Q_sca, accurate to the quadrature error."""
    from .dda import effective_radius

    th, ph, w = scattering_directions(x, eta)
    n_lab, _, _ = lab_direction_basis(th, ph)
    n_tf = n_lab @ np.asarray(lab_axes, dtype=np.float64)
    phase = np.exp(-1j * k * (n_tf @ np.asarray(r).T))
    F = phase @ np.asarray(P, dtype=np.complex128)
    Fperp = F - n_tf * np.sum(n_tf * F, axis=1)[:, None]
    dC = k ** 4 * np.sum(np.abs(Fperp) ** 2, axis=1)
    return float(np.sum(w * dC) / (np.pi * effective_radius(len(r)) ** 2))


def quadrature_directions_tf(x, eta, lab_axes):
    """Target-frame directions and solid-angle weights of the eta-controlled
    scattering-direction set ("Averaging over Scattering Directions")."""
    th, ph, w = scattering_directions(x, eta)
    n_lab, _, _ = lab_direction_basis(th, ph)
    return n_lab @ np.asarray(lab_axes, dtype=np.float64), w


def differential_cross_section(r, k, P, n_tf):
    """dC_sca/dOmega = k^4 |sum_j (P_j - n (n . P_j)) exp(-i k n . r_j)|^2 for
    each direction n (|E_0| = 1)."""
    phase = np.exp(-1j * k * (np.asarray(n_tf) @ np.asarray(r, dtype=np.float64).T))
    F = phase @ np.asarray(P, dtype=np.complex128)
    Fperp = F - n_tf * np.sum(n_tf * F, axis=1)[:, None]
    return k ** 4 * np.sum(np.abs(Fperp) ** 2, axis=1)


def scattering_moments(r, k, E, P, ainv, khat, n_tf, w):
    """Efficiencies and moments of one solution, Q = C / (pi a_eff^2):

    * Q_pha from C_pha = 2 pi k Re sum_j E_j^* . P_j (the phase-shift cross
      section of Draine 1988: a dilute medium of targets retards the phase by
      n_t C_pha per unit length; for a dipole alpha it is 2 pi k Re(alpha));
    * Q_bk = (dC_sca/dOmega at n = -khat) / (pi a_eff^2);
    * with the quadrature directions n_tf and weights w ("Averaging over
      Scattering Directions"): Q_sca from the quadrature, Q_sca g = sum w dC n
      / (pi a_eff^2) (target frame), <cos theta> = g . khat and
      <cos^2 theta> = sum w dC (n . khat)^2 / C_sca, normalized by
      C_sca = C_ext - C_abs (reading; the guide's printed worked example has
      g(1) = Q_sca g(1) / Q_sca with that Q_sca);
    * Q_pr = Q_ext khat - Q_sca g (section "Calculation of <cos theta>,
      Radiative Force, and Radiation Torque").

    Returns a dict of these values.
    """
    from .dda import cross_sections, effective_radius

    n = len(r)
    area = np.pi * effective_radius(n) ** 2
    khat = np.asarray(khat, dtype=np.float64)
    qext, qabs, qsca = cross_sections(k, E, P, ainv, n)
    qpha = 2.0 * np.pi * k * np.sum(np.real(np.conj(E) * P)) / area
    qbk = float(differential_cross_section(r, k, P, -khat[None, :])[0] / area)
    dC = differential_cross_section(r, k, P, n_tf)
    qsca_quad = float(np.sum(w * dC) / area)
    qg = np.sum((w * dC)[:, None] * n_tf, axis=0) / area
    cosm = float(np.dot(qg, khat) / qsca)
    cos2 = float(np.sum(w * dC * (n_tf @ khat) ** 2) / area / qsca)
    return {"Qext": qext, "Qabs": qabs, "Qsca": qsca, "Qpha": float(qpha), "Qbk": qbk,
            "Qsca_quad": qsca_quad, "Qsca_g": qg, "cos": cosm, "cos2": cos2, "Qpr": qext * khat - qg}
