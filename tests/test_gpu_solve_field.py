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
