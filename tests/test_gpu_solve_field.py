"""dda_solve_field: A P = E for caller-supplied incident fields, through the
C ABI, against dda_solve (plane waves) and the oracle's dense solve (any
field).  Inputs are seeded and synthetic; expected values come from
``oracle/``."""
import numpy as np
import pytest

import synth
from oracle import dda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1002_1505_amd as P

    c = P.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _target(ctx, kind):
    import paper_1002_1505_amd as P

    occ = synth.ellipsoid_occupancy((10, 9, 8), (9.4, 8.2, 7.3))
    m, kd = 1.55 + 0.12j, 0.42
    kinds = {dda.ALPHA_CM: P.DDA_ALPHA_CM, dda.ALPHA_LDR: P.DDA_ALPHA_LDR}
    ctx.set_target(occ, [m], kd, kinds[kind])
    r, comp, _ = dda.sites_from_occupancy(occ)
    return r, comp, m, kd


def test_plane_wave_field_reproduces_solve(ctx):
    """E given as the plane wave itself: the same solution as dda_solve."""
    import paper_1002_1505_amd as P

    r, comp, m, kd = _target(ctx, dda.ALPHA_LDR)
    kh, es, L = dda.waves_for_orientation(0.3, 0.9, 0.5)
    E = [dda.incident_field(r, kd, kh, e) for e in es]
    Pw, sw, _ = ctx.solve([kh, kh], es, prec=P.DDA_SOLVE_FP64, tol=1e-11)
    qw = ctx.cross_sections(2)
    Pf, sf, _ = ctx.solve([kh, kh], es, prec=P.DDA_SOLVE_FP64, tol=1e-11, e_inc=E)
    qf = ctx.cross_sections(2)
    for l in range(2):
        assert sf[l]["rel_resid"] <= 1e-11
        assert _rel(Pf[l], Pw[l]) < 1e-9
    assert np.allclose(qf, qw, rtol=1e-9, atol=0)


@pytest.mark.parametrize("kind", [dda.ALPHA_CM, dda.ALPHA_LDR])
def test_random_field_vs_oracle(ctx, kind):
    """A seeded random complex field: P against the oracle's dense solve with
    the same 1/alpha (which the waves select), and the efficiencies of
    that field."""
    import paper_1002_1505_amd as P

    r, comp, m, kd = _target(ctx, kind)
    kh, es, L = dda.waves_for_orientation(1.1, 0.4, 2.0)
    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 17)
    E = [rng.standard_normal((len(r), 3)) + 1j * rng.standard_normal((len(r), 3)) for _ in range(2)]
    Pf, sf, _ = ctx.solve([kh, kh], es, prec=P.DDA_SOLVE_FP64, tol=1e-11, e_inc=E)
    q = ctx.cross_sections(2)
    for l in range(2):
        ainv = dda.site_inverse_polarizability(comp, [m], kd, kind, kh, es[l])
        want = dda.solve_dense(r, kd, ainv, E[l])
        assert sf[l]["rel_resid"] <= 1e-11
        assert _rel(Pf[l], want) < 1e-9, l
        qe, qa, qs = dda.cross_sections(kd, E[l], want, ainv)
        assert np.allclose(q[l], [qe, qa, qs], rtol=1e-8, atol=1e-12), (l, q[l], (qe, qa, qs))


def test_fp32_refine_field_reaches_the_residual(ctx):
    """FP32 matvec with FP64 refinement on a caller field: the oracle's own
    residual ||E - A P|| / ||E|| of the returned P is at the tolerance."""
    import paper_1002_1505_amd as P

    r, comp, m, kd = _target(ctx, dda.ALPHA_LDR)
    kh, es, L = dda.waves_for_orientation(0.0, 1.3, 0.7)
    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 19)
    E = [rng.standard_normal((len(r), 3)) + 1j * rng.standard_normal((len(r), 3)) for _ in range(2)]
    Pf, sf, _ = ctx.solve([kh, kh], es, prec=P.DDA_SOLVE_FP32_REFINE, tol=1e-6, e_inc=E)
    for l in range(2):
        ainv = dda.site_inverse_polarizability(comp, [m], kd, dda.ALPHA_LDR, kh, es[l])
        res = np.linalg.norm(E[l] - dda.matvec_direct(r, kd, ainv, Pf[l])) / np.linalg.norm(E[l])
        assert sf[l]["rel_resid"] <= 1e-6 and res <= 1.5e-6, (l, res)


def test_solve_field_rejects_a_missing_field(ctx):
    import ctypes as C

    import paper_1002_1505_amd as P
    from paper_1002_1505_amd import _lib as L

    _target(ctx, dda.ALPHA_CM)
    kh, es, L_ = dda.waves_for_orientation(0.0, 0.0, 0.0)
    arr = (L.dda_wave * 1)()
    arr[0].khat[:] = list(kh)
    for j in range(3):
        arr[0].e0[2 * j], arr[0].e0[2 * j + 1] = es[0][j].real, es[0][j].imag
    opts = L.dda_solve_opts(tol=1e-5, max_iter=100, guess=P.DDA_GUESS_ZERO, prec=P.DDA_SOLVE_FP64)
    st = ctx.lib.dda_solve_field(ctx.h, 1, arr, C.byref(opts), None, None, None, None)
    assert st == L.DDA_ERR_INVALID_ARG


class _DeviceBuffer:
    """Device memory from the HIP runtime the library itself uses (the
    library's soname, so the process has one runtime)."""

    def __init__(self, nbytes):
        import ctypes as C

        from paper_1002_1505_amd import _lib as L

        L.load()
        self.hip = C.CDLL("libamdhip64.so.7")
        self.n = nbytes
        self.p = C.c_void_p()
        assert self.hip.hipMalloc(C.byref(self.p), C.c_size_t(nbytes)) == 0

    def upload(self, a):
        import ctypes as C

        a = np.ascontiguousarray(a)
        assert a.nbytes == self.n
        assert self.hip.hipMemcpy(self.p, C.c_void_p(a.ctypes.data), C.c_size_t(self.n), 1) == 0  # host to device

    def download(self, dtype):
        import ctypes as C

        out = np.empty(self.n // np.dtype(dtype).itemsize, dtype=dtype)
        assert self.hip.hipMemcpy(C.c_void_p(out.ctypes.data), self.p, C.c_size_t(self.n), 2) == 0  # device to host
        return out

    def free(self):
        self.hip.hipFree(self.p)


def test_device_pointer_buffers_match_host_buffers(ctx):
    """DDA_DEVICE_PTRS: the caller's field, guess and solution as device
    buffers give the same bits as host buffers."""
    import ctypes as C

    import paper_1002_1505_amd as P
    from paper_1002_1505_amd import _lib as L

    r, comp, m, kd = _target(ctx, dda.ALPHA_LDR)
    kh, es, L_ = dda.waves_for_orientation(0.6, 2.1, 1.4)
    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 23)
    E = [rng.standard_normal((len(r), 3)) + 1j * rng.standard_normal((len(r), 3)) for _ in range(2)]
    Ph, sh, _ = ctx.solve([kh, kh], es, prec=P.DDA_SOLVE_FP64, tol=1e-10, e_inc=E)
    eh = np.ascontiguousarray(np.concatenate([e.reshape(-1) for e in E]))
    e_d, p_d, g_d, p2 = (_DeviceBuffer(eh.nbytes) for _ in range(4))
    try:
        e_d.upload(eh)
        arr, n = P._waves([kh, kh], es, None)
        stats = (L.dda_solve_stats * 2)()
        opts = L.dda_solve_opts(tol=1e-10, max_iter=1000, guess=P.DDA_GUESS_ZERO, prec=P.DDA_SOLVE_FP64,
                                flags=L.DDA_DEVICE_PTRS)
        st = ctx.lib.dda_solve_field(ctx.h, 2, arr, C.byref(opts), e_d.p, None, p_d.p, stats)
        assert st == 0, ctx.last_error()
        Pd = p_d.download(np.complex128).reshape(2, len(r), 3)
        for l in range(2):
            assert stats[l].iters == sh[l]["iters"]
            assert np.array_equal(Pd[l], Ph[l]), l
        # the solution itself as a device guess: converged before any iteration
        g_d.upload(Pd)
        opts.guess = P.DDA_GUESS_USER
        st = ctx.lib.dda_solve_field(ctx.h, 2, arr, C.byref(opts), e_d.p, g_d.p, p2.p, stats)
        assert st == 0, ctx.last_error()
        assert all(stats[l].iters == 0 for l in range(2))
        assert np.array_equal(p2.download(np.complex128).reshape(2, len(r), 3), Pd)
    finally:
        for b in (e_d, p_d, g_d, p2):
            b.free()
