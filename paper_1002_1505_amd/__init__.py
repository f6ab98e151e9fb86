"""Python binding of the MI355X DDA solver library (``libdda.so``).

Thin argument marshalling over the C ABI of ``include/dda.h``: every step of
the solve runs in the library's HIP kernels.  Arrays are numpy arrays on the
host, or torch CUDA tensors (device pointers) where noted.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import (DDA_ALPHA_CM, DDA_ALPHA_CM_RR, DDA_ALPHA_LDR, DDA_DEVICE_PTRS, DDA_FP32, DDA_FP64,  # noqa: F401
                   DDA_GUESS_NN, DDA_GUESS_PREV, DDA_GUESS_PREV_SHIFT, DDA_GUESS_PROJECT, DDA_GUESS_USER,
                   DDA_GUESS_ZERO, DDA_NO_FALLBACK, DDA_NO_GRAPH,
                   DDA_SOLVE_FP32_REFINE, DDA_SOLVE_FP64, DDA_SOLVER_BICGSTAB, DDA_SOLVER_BICGSTAB2,
                   DDA_WARN_MKD_GE_1, DDA_WARN_NOT_CONVERGED)

__all__ = ["Context", "DDAError", "lab_frame", "mueller", "orientation_waves", "scattering_frame", "load_library"]


class DDAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dda status {status}: {msg}")
        self.status = status


def load_library():
    return L.load()


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(ctx, status):
    if status < 0:
        lib = L.load()
        msg = lib.dda_last_error(ctx).decode() if ctx else "error"
        raise DDAError(status, msg)
    return status


def _waves(khat, e0, targets):
    khat = np.asarray(khat, dtype=np.float64).reshape(-1, 3)
    e0 = np.asarray(e0, dtype=np.complex128).reshape(-1, 3)
    n = len(khat)
    if targets is None:
        targets = np.zeros(n, dtype=np.int32)
    targets = np.broadcast_to(np.asarray(targets, dtype=np.int32), (n,))
    arr = (L.dda_wave * n)()
    for i in range(n):
        for j in range(3):
            arr[i].khat[j] = khat[i, j]
            arr[i].e0[2 * j] = e0[i, j].real
            arr[i].e0[2 * j + 1] = e0[i, j].imag
        arr[i].target = int(targets[i])
    return arr, n


class Context:
    """A solver context on one GPU (dda_create / dda_destroy)."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self.lib = L.load()
        h = C.c_void_p()
        st = self.lib.dda_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None)
        if st < 0:
            raise DDAError(st, "dda_create failed: " + self.lib.dda_last_error(None).decode())
        self.h = h
        self.n_sites = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.dda_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def last_error(self) -> str:
        return self.lib.dda_last_error(self.h).decode()

    # -- targets ---------------------------------------------------------
    def _target_args(self, occ, m, kd, alpha_kind, origin):
        occ = np.ascontiguousarray(occ, dtype=np.uint8)
        if occ.ndim != 3:
            raise ValueError("occupancy must be 3-D (n3, n2, n1), x fastest")
        dims = (C.c_int32 * 3)(occ.shape[2], occ.shape[1], occ.shape[0])
        mm = np.atleast_1d(np.asarray(m, dtype=np.complex128))
        marr = np.ascontiguousarray(np.stack([mm.real, mm.imag], axis=1).reshape(-1))
        org = None if origin is None else np.ascontiguousarray(origin, dtype=np.float64)
        return occ, dims, mm, marr, org

    def set_target(self, occ, m, kd, alpha_kind=DDA_ALPHA_LDR, origin=None) -> int:
        occ, dims, mm, marr, org = self._target_args(occ, m, kd, alpha_kind, origin)
        st = self.lib.dda_set_target(self.h, dims, occ.ctypes.data, len(mm), _dptr(marr), float(kd), int(alpha_kind),
                                     None if org is None else _dptr(org))
        _check(self.h, st)
        self.n_sites = {0: self.target_info(0)[0]}
        return st

    def add_target(self, occ, m, kd, alpha_kind=DDA_ALPHA_LDR, origin=None) -> int:
        occ, dims, mm, marr, org = self._target_args(occ, m, kd, alpha_kind, origin)
        tid = C.c_int32()
        st = self.lib.dda_add_target(self.h, dims, occ.ctypes.data, len(mm), _dptr(marr), float(kd), int(alpha_kind),
                                     None if org is None else _dptr(org), C.byref(tid))
        _check(self.h, st)
        self.n_sites[tid.value] = self.target_info(tid.value)[0]
        return tid.value

    def target_info(self, target: int = 0):
        n = C.c_int64()
        a = C.c_double()
        _check(self.h, self.lib.dda_target_info(self.h, int(target), C.byref(n), C.byref(a)))
        return int(n.value), float(a.value)

    def set_anisotropic(self, comp, m3, angles, target: int = 0) -> int:
        """Composition `comp` (1-based) anisotropic: principal refractive
        indices m3 (3 complex) along the Dielectric Frame axes, frame angles
        (Theta_DF, Phi_DF, beta_DF) in radians (dda_set_anisotropic)."""
        mm = np.asarray(m3, dtype=np.complex128).reshape(3)
        marr = np.ascontiguousarray(np.stack([mm.real, mm.imag], axis=1).reshape(-1))
        ang = np.ascontiguousarray(np.asarray(angles, dtype=np.float64).reshape(3))
        return _check(self.h, self.lib.dda_set_anisotropic(self.h, int(target), int(comp), _dptr(marr), _dptr(ang)))

    def build_green_fft(self, prec=DDA_FP32 | DDA_FP64):
        return _check(self.h, self.lib.dda_build_green_fft(self.h, int(prec)))

    def inverse_polarizability(self, khat, e0, target: int = 0):
        arr, _ = _waves(khat, e0, [target])
        n_comp = 256
        out = np.zeros(2 * n_comp)
        _check(self.h, self.lib.dda_inverse_polarizability(self.h, int(target), arr, _dptr(out)))
        return out

    # -- solve -----------------------------------------------------------
    def solve(self, khat, e0, targets=None, tol=1e-5, max_iter=1000, guess=DDA_GUESS_ZERO,
              prec=DDA_SOLVE_FP32_REFINE, p0=None, want_p=True, flags=0, graph_iters=0, history=0, e_inc=None,
              restart_every=0, solver=DDA_SOLVER_BICGSTAB):
        """Solve A P = E_inc for each wave; returns (P or None, stats list, status).

        P is a list of (N_t, 3) complex128 arrays (one per wave).  With e_inc
        (a list of (N_t, 3) complex128 fields, one per wave) the right-hand
        sides are those fields (dda_solve_field); the waves then select the
        targets and polarizabilities only."""
        arr, n = _waves(khat, e0, targets)
        opts = L.dda_solve_opts(tol=tol, max_iter=max_iter, guess=guess, prec=prec, flags=flags,
                                graph_iters=graph_iters, history=history, restart_every=restart_every,
                                solver=solver)
        tg = [arr[i].target for i in range(n)]
        sizes = [self.n_sites.get(t, 0) for t in tg]  # unknown ids: the library rejects the call
        p0buf = None
        if p0 is not None:
            p0buf = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.complex128).reshape(-1) for p in p0]))
        pout = np.zeros(3 * sum(sizes), dtype=np.complex128) if want_p else None
        stats = (L.dda_solve_stats * n)()
        if e_inc is None:
            st = self.lib.dda_solve(self.h, n, arr, C.byref(opts),
                                    None if p0buf is None else p0buf.ctypes.data,
                                    None if pout is None else pout.ctypes.data, stats)
        else:
            ebuf = np.ascontiguousarray(np.concatenate([np.asarray(e, dtype=np.complex128).reshape(-1)
                                                        for e in e_inc]))
            if ebuf.size != 3 * sum(sizes):
                raise ValueError("e_inc: one (N_t, 3) field per wave")
            st = self.lib.dda_solve_field(self.h, n, arr, C.byref(opts), ebuf.ctypes.data,
                                          None if p0buf is None else p0buf.ctypes.data,
                                          None if pout is None else pout.ctypes.data, stats)
        _check(self.h, st)
        P = None
        if want_p:
            P, off = [], 0
            for s in sizes:
                P.append(pout[off:off + 3 * s].reshape(s, 3))
                off += 3 * s
        sl = [dict(iters=s.iters, matvecs=s.matvecs, outer=s.outer, status=s.status, rel_resid=s.rel_resid,
                   guess_resid=s.guess_resid) for s in stats]
        return P, sl, st

    def matvec(self, x, target: int = 0, ainv=None, prec=DDA_FP64):
        """y = A x for x of shape (nrhs, N, 3) complex128."""
        x = np.ascontiguousarray(x, dtype=np.complex128)
        if x.ndim == 2:
            x = x[None]
        nrhs = x.shape[0]
        y = np.zeros_like(x)
        a = None
        if ainv is not None:
            a = np.ascontiguousarray(np.asarray(ainv, dtype=np.complex128).reshape(nrhs, -1))
            a = np.ascontiguousarray(np.stack([a.real, a.imag], axis=-1).reshape(-1))
        _check(self.h, self.lib.dda_matvec(self.h, int(target), nrhs, None if a is None else _dptr(a),
                                           x.ctypes.data, y.ctypes.data, int(prec), 0))
        return y

    def cross_sections(self, nrhs: int):
        q = np.zeros(3 * nrhs)
        _check(self.h, self.lib.dda_cross_sections(self.h, int(nrhs), _dptr(q)))
        return q.reshape(nrhs, 3)

    def cross_sections_phi(self, coeffs):
        """Efficiencies of combined polarization pairs (dda_cross_sections_phi):
        coeffs (npairs, ncomb, 2, 2) complex; returns (npairs, ncomb, 2, 3)."""
        c = np.asarray(coeffs, dtype=np.complex128)
        npairs, ncomb = c.shape[0], c.shape[1]
        cc = np.ascontiguousarray(np.stack([c.real, c.imag], axis=-1).reshape(-1))
        q = np.zeros(npairs * ncomb * 2 * 3)
        _check(self.h, self.lib.dda_cross_sections_phi(self.h, int(npairs), int(ncomb), _dptr(cc), _dptr(q)))
        return q.reshape(npairs, ncomb, 2, 3)

    MOMENT_KEYS = ("Qpha", "Qbk", "Qsca_quad", "Qsca_g", "cos", "cos2", "Qpr")

    def scattering_moments(self, nrhs: int, n_tf, w):
        """Per rhs dict of Q_pha, Q_bk, quadrature Q_sca, Q_sca g (3), <cos>,
        <cos^2>, Q_pr (3) (dda_scattering_moments)."""
        n_tf = np.ascontiguousarray(n_tf, dtype=np.float64).reshape(-1, 3)
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
        out = np.zeros(nrhs * 11)
        _check(self.h, self.lib.dda_scattering_moments(self.h, int(nrhs), len(w), _dptr(n_tf), _dptr(w), _dptr(out)))
        out = out.reshape(nrhs, 11)
        return [dict(Qpha=o[0], Qbk=o[1], Qsca_quad=o[2], Qsca_g=o[3:6].copy(), cos=o[6], cos2=o[7],
                     Qpr=o[8:11].copy()) for o in out]

    def amplitudes(self, nrhs: int, n_tf, e_tf):
        n_tf = np.ascontiguousarray(n_tf, dtype=np.float64).reshape(-1, 3)
        e_tf = np.ascontiguousarray(e_tf, dtype=np.float64).reshape(-1, 6)
        ndir = len(n_tf)
        f = np.zeros(nrhs * ndir * 2 * 2)
        _check(self.h, self.lib.dda_amplitudes(self.h, int(nrhs), ndir, _dptr(n_tf), _dptr(e_tf), _dptr(f)))
        f = f.reshape(nrhs, ndir, 2, 2)
        return f[..., 0] + 1j * f[..., 1]

    def amplitudes_per_rhs(self, nrhs: int, n_tf, e_tf):
        """Amplitudes with a direction set per rhs: n_tf (nrhs, ndir, 3), e_tf
        (nrhs, ndir, 6); returns (nrhs, ndir, 2) complex (dda_amplitudes_per_rhs)."""
        n_tf = np.ascontiguousarray(n_tf, dtype=np.float64).reshape(nrhs, -1, 3)
        ndir = n_tf.shape[1]
        e_tf = np.ascontiguousarray(e_tf, dtype=np.float64).reshape(nrhs, ndir, 6)
        f = np.zeros(nrhs * ndir * 2 * 2)
        _check(self.h, self.lib.dda_amplitudes_per_rhs(self.h, int(nrhs), ndir, _dptr(n_tf), _dptr(e_tf), _dptr(f)))
        f = f.reshape(nrhs, ndir, 2, 2)
        return f[..., 0] + 1j * f[..., 1]

    def near_field(self, nrhs: int, points, want_b=True):
        """Total E (and B) at points (npts, 3) in the target frame, lattice
        units from the target origin, for every rhs of the last solve
        (dda_near_field); returns (E, B) of shape (nrhs, npts, 3) complex."""
        pts = np.ascontiguousarray(np.asarray(points, dtype=np.float64).reshape(-1, 3))
        n = len(pts)
        E = np.zeros(nrhs * n * 6)
        B = np.zeros(nrhs * n * 6) if want_b else None
        _check(self.h, self.lib.dda_near_field(self.h, int(nrhs), n, _dptr(pts), _dptr(E),
                                               None if B is None else _dptr(B)))
        E = E.reshape(nrhs, n, 3, 2)
        E = E[..., 0] + 1j * E[..., 1]
        if B is not None:
            B = B.reshape(nrhs, n, 3, 2)
            B = B[..., 0] + 1j * B[..., 1]
        return E, B

    def last_timing(self):
        a, b, t, g = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        self.lib.dda_last_timing(self.h, C.byref(a), C.byref(b), C.byref(t))
        self.lib.dda_last_guess_ms(self.h, C.byref(g))
        return dict(ms_mv32=a.value, ms_mv64=b.value, ms_total=t.value, ms_guess=g.value)

    def profile_matvec(self, target=0, nrhs=1, prec=DDA_FP32, reps=10):
        ms = np.zeros(3)
        by = np.zeros(3)
        _check(self.h, self.lib.dda_profile_matvec(self.h, int(target), int(nrhs), int(prec), int(reps), _dptr(ms),
                                                   _dptr(by)))
        return ms, by

    def get_shape(self, target=0, prec=DDA_FP32):
        out = (C.c_int32 * 8)()
        _check(self.h, self.lib.dda_get_shape(self.h, int(target), int(prec), out))
        keys = ["fused", "nth_plane", "nth_z", "tx", "lines_tl", "nth_lines", "ct", "zrb"]
        return dict(zip(keys, list(out)))

    def set_shape(self, shape: dict, target=0, prec=DDA_FP32):
        keys = ["fused", "nth_plane", "nth_z", "tx", "lines_tl", "nth_lines", "ct", "zrb"]
        arr = (C.c_int32 * 8)(*[int(shape[k]) for k in keys])
        _check(self.h, self.lib.dda_set_shape(self.h, int(target), int(prec), arr))

    def autotune(self, nrhs_hint=2, cache_path=None):
        return _check(self.h, self.lib.dda_autotune(self.h, int(nrhs_hint),
                                                    None if cache_path is None else cache_path.encode()))


def lab_frame(beta, theta, phi, a1=None, a2=None):
    lib = L.load()
    out = np.zeros(9)
    a1 = None if a1 is None else np.ascontiguousarray(a1, dtype=np.float64)
    a2 = None if a2 is None else np.ascontiguousarray(a2, dtype=np.float64)
    st = lib.dda_lab_frame(float(beta), float(theta), float(phi), None if a1 is None else _dptr(a1),
                           None if a2 is None else _dptr(a2), _dptr(out))
    if st < 0:
        raise DDAError(st, "dda_lab_frame")
    return out.reshape(3, 3)


def orientation_waves(beta, theta, phi, e01=None, a1=None, a2=None, target=0):
    """(khat (2, 3), e0 (2, 3) complex) of the two incident polarizations of an
    orientation, in the target frame (dda_orientation_waves)."""
    lib = L.load()
    out = (L.dda_wave * 2)()
    e = None
    if e01 is not None:
        ev = np.asarray(e01, dtype=np.complex128)
        e = np.ascontiguousarray(np.stack([ev.real, ev.imag], axis=1).reshape(-1))
    a1 = None if a1 is None else np.ascontiguousarray(a1, dtype=np.float64)
    a2 = None if a2 is None else np.ascontiguousarray(a2, dtype=np.float64)
    st = lib.dda_orientation_waves(float(beta), float(theta), float(phi), None if a1 is None else _dptr(a1),
                                   None if a2 is None else _dptr(a2), None if e is None else _dptr(e), int(target), out)
    if st < 0:
        raise DDAError(st, "dda_orientation_waves")
    kh = np.array([[out[w].khat[i] for i in range(3)] for w in range(2)])
    e0 = np.array([[out[w].e0[2 * i] + 1j * out[w].e0[2 * i + 1] for i in range(3)] for w in range(2)])
    return kh, e0


def scattering_quadrature(x, eta, lab_axes):
    """(n_tf (ndir, 3), w (ndir,)) of dda_scattering_quadrature."""
    lib = L.load()
    La = np.ascontiguousarray(lab_axes, dtype=np.float64).reshape(-1)
    nd = C.c_int32()
    st = lib.dda_scattering_quadrature(float(x), float(eta), _dptr(La), 0, C.byref(nd), None, None)
    if st < 0:
        raise DDAError(st, "dda_scattering_quadrature")
    n_tf, w = np.zeros(3 * nd.value), np.zeros(nd.value)
    st = lib.dda_scattering_quadrature(float(x), float(eta), _dptr(La), nd.value, C.byref(nd), _dptr(n_tf), _dptr(w))
    if st < 0:
        raise DDAError(st, "dda_scattering_quadrature")
    return n_tf.reshape(-1, 3), w


def orientation_samples(lims, counts):
    """(beta, theta, phi, weight (nb, nt, np)) of dda_orientation_samples;
    lims = (BETAMI, BETAMX, THETMI, THETMX, PHIMIN, PHIMAX) in radians."""
    lib = L.load()
    lm = np.ascontiguousarray(lims, dtype=np.float64)
    n = (C.c_int32 * 3)(*[int(v) for v in counts])
    b, t, p = np.zeros(n[0]), np.zeros(n[1]), np.zeros(n[2])
    w = np.zeros(n[0] * n[1] * n[2])
    st = lib.dda_orientation_samples(_dptr(lm), n, _dptr(b), _dptr(t), _dptr(p), _dptr(w))
    if st < 0:
        raise DDAError(st, "dda_orientation_samples")
    return b, t, p, w.reshape(n[0], n[1], n[2])


def phi_coefficients(beta, theta, phi_ref, phis, e01=None, a1=None, a2=None):
    """c (nphi, 2, 2) complex of dda_phi_coefficients."""
    lib = L.load()
    ph = np.ascontiguousarray(phis, dtype=np.float64).reshape(-1)
    e = None
    if e01 is not None:
        ev = np.asarray(e01, dtype=np.complex128)
        e = np.ascontiguousarray(np.stack([ev.real, ev.imag], axis=1).reshape(-1))
    a1 = None if a1 is None else np.ascontiguousarray(a1, dtype=np.float64)
    a2 = None if a2 is None else np.ascontiguousarray(a2, dtype=np.float64)
    out = np.zeros(len(ph) * 8)
    st = lib.dda_phi_coefficients(float(beta), float(theta), float(phi_ref), len(ph), _dptr(ph),
                                  None if a1 is None else _dptr(a1), None if a2 is None else _dptr(a2),
                                  None if e is None else _dptr(e), _dptr(out))
    if st < 0:
        raise DDAError(st, "dda_phi_coefficients")
    out = out.reshape(len(ph), 2, 2, 2)
    return out[..., 0] + 1j * out[..., 1]


def scattering_frame(theta, phi, lab_axes):
    """(n_tf (ndir, 3), e_tf (ndir, 6)) for lab-frame scattering angles (dda_scattering_frame)."""
    lib = L.load()
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
    ph = np.ascontiguousarray(np.broadcast_to(phi, th.shape), dtype=np.float64)
    La = np.ascontiguousarray(lab_axes, dtype=np.float64).reshape(-1)
    n = np.zeros((len(th), 3))
    e = np.zeros((len(th), 6))
    st = lib.dda_scattering_frame(len(th), _dptr(th), _dptr(ph), _dptr(La), _dptr(n), _dptr(e))
    if st < 0:
        raise DDAError(st, "dda_scattering_frame")
    return n, e


def polarization(mueller, k, stokes_in=(1.0, 0.0, 0.0, 0.0)):
    """(ndir, 4): dC_sca/dOmega parallel and perpendicular to the scattering
    plane and in total for the incident Stokes vector, and the linear
    polarization P for unpolarized incidence (dda_polarization); mueller is
    (ndir, 4, 4) as returned by mueller()."""
    lib = L.load()
    mu = np.ascontiguousarray(np.asarray(mueller, dtype=np.float64).reshape(-1, 16))
    s = np.ascontiguousarray(np.asarray(stokes_in, dtype=np.float64).reshape(4))
    out = np.zeros((len(mu), 4))
    st = lib.dda_polarization(len(mu), _dptr(mu), float(k), _dptr(s), _dptr(out))
    if st != 0:
        raise DDAError(st, "dda_polarization: bad arguments")
    return out


def mueller(f, phi, e01, e02):
    """S_1..S_4 (ndir, 4) and Mueller (ndir, 4, 4) from f[dir, m, l]."""
    lib = L.load()
    f = np.ascontiguousarray(f, dtype=np.complex128)
    ndir = f.shape[0]
    fb = np.ascontiguousarray(np.stack([f.real, f.imag], axis=-1).reshape(-1))
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    e1 = np.asarray(e01, dtype=np.complex128)
    e2 = np.asarray(e02, dtype=np.complex128)
    e1b = np.ascontiguousarray(np.stack([e1.real, e1.imag], axis=-1).reshape(-1))
    e2b = np.ascontiguousarray(np.stack([e2.real, e2.imag], axis=-1).reshape(-1))
    S = np.zeros(ndir * 8)
    M = np.zeros(ndir * 16)
    st = lib.dda_mueller(ndir, _dptr(fb), _dptr(ph), _dptr(e1b), _dptr(e2b), _dptr(S), _dptr(M))
    if st < 0:
        raise DDAError(st, "dda_mueller")
    S = S.reshape(ndir, 4, 2)
    return S[..., 0] + 1j * S[..., 1], M.reshape(ndir, 4, 4)


class Net:
    """Learned initial-guess network (dda_nn_*)."""

    def __init__(self, ctx: Context, width=32, depth=6, seed=1):
        self.lib = L.load()
        self.ctx = ctx
        h = C.c_void_p()
        cfg = L.dda_nn_config(width=width, depth=depth, seed=seed)
        st = self.lib.dda_nn_create(ctx.h, C.byref(cfg), C.byref(h))
        if st < 0:
            raise DDAError(st, "dda_nn_create failed")
        self.h = h
        self.depth = depth

    def close(self):
        if getattr(self, "h", None):
            self.lib.dda_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self) -> int:
        return int(self.lib.dda_nn_num_params(self.h))

    @property
    def num_samples(self) -> int:
        return int(self.lib.dda_nn_num_samples(self.h))

    def layers(self):
        out = (C.c_int32 * (3 * self.depth))()
        _check(None, self.lib.dda_nn_layer_info(self.h, out))
        return [(out[3 * i], out[3 * i + 1], out[3 * i + 2]) for i in range(self.depth)]

    def get_params(self):
        flat = np.zeros(self.num_params, dtype=np.float32)
        _check(None, self.lib.dda_nn_get_params(self.h, flat.ctypes.data_as(C.POINTER(C.c_float))))
        return self._unflat(flat)

    def set_params(self, params):
        flat = np.ascontiguousarray(np.concatenate([np.concatenate([w.reshape(-1), b.reshape(-1)]) for w, b in params]),
                                    dtype=np.float32)
        assert flat.size == self.num_params
        _check(None, self.lib.dda_nn_set_params(self.h, flat.ctypes.data_as(C.POINTER(C.c_float))))

    def _unflat(self, flat):
        out, off = [], 0
        for cin, cout, d in self.layers():
            n = 27 * cin * cout
            out.append((flat[off:off + n].reshape(27, cin, cout), flat[off + n:off + n + cout]))
            off += n + cout
        return out

    def attach(self):
        _check(self.ctx.h, self.lib.dda_set_guess_model(self.ctx.h, self.h))

    def record(self):
        _check(self.ctx.h, self.lib.dda_nn_record(self.ctx.h, self.h))

    def train(self, epochs=1, batch=4, lr=1e-3, weight_decay=0.0):
        o = L.dda_nn_train_opts(epochs=epochs, batch=batch, lr=lr, weight_decay=weight_decay)
        loss = C.c_double()
        _check(self.ctx.h, self.lib.dda_nn_train(self.ctx.h, self.h, C.byref(o), C.byref(loss)))
        return loss.value

    def save(self, path):
        _check(None, self.lib.dda_nn_save(self.h, path.encode()))

    def load(self, path):
        _check(None, self.lib.dda_nn_load(self.h, path.encode()))

    def profile(self, D=64, ns=2, reps=10):
        """(ms per forward, ms per parameter-gradient pass, forward GFLOP) on ns
        device-resident D^3 samples."""
        a, b, g = C.c_double(), C.c_double(), C.c_double()
        _check(None, self.lib.dda_nn_profile(self.h, int(D), int(ns), int(reps), C.byref(a), C.byref(b), C.byref(g)))
        return a.value, b.value, g.value

    def forward_backward(self, x, target=None, mask=None, nout=6):
        """x: (ns, D, D, D, 16) float32; returns (out, grads as [(dW, db)], loss)."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        ns, D = x.shape[0], x.shape[1]
        out = np.zeros((ns, D, D, D, 16), dtype=np.float32)
        fp = lambda a: a.ctypes.data_as(C.POINTER(C.c_float))
        if target is None:
            _check(None, self.lib.dda_nn_forward_backward(self.h, ns, D, fp(x), None, None, nout, fp(out), None, None))
            return out, None, None
        t = np.ascontiguousarray(target, dtype=np.float32)
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        g = np.zeros(self.num_params, dtype=np.float32)
        loss = C.c_double()
        _check(None, self.lib.dda_nn_forward_backward(self.h, ns, D, fp(x), fp(t), m.ctypes.data, nout, fp(out), fp(g),
                                                      C.byref(loss)))
        return out, self._unflat(g), loss.value
