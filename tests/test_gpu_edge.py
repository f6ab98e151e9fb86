"""Edge cases of the C ABI on the GPU: rejected inputs return errors (and
leave the context usable), the smallest target reduces to the isolated-dipole
closed form, and a wide batch of right-hand sides matches the oracle."""
import ctypes as C

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


def test_rejected_targets_leave_context_usable(ctx):
    import paper_1002_1505_amd as P

    with pytest.raises(P.DDAError):  # no occupied site
        ctx.set_target(np.zeros((4, 4, 4), np.uint8), [1.5 + 0.1j], 0.3)
    with pytest.raises(P.DDAError):  # composition 2 of 1
        ctx.set_target(2 * np.ones((4, 4, 4), np.uint8), [1.5 + 0.1j], 0.3)
    with pytest.raises(P.DDAError):  # 7 does not factor into 2, 3, 5
        ctx.set_target(np.ones((7, 8, 8), np.uint8), [1.5 + 0.1j], 0.3)
    with pytest.raises(P.DDAError):  # k d must be positive
        ctx.set_target(np.ones((4, 4, 4), np.uint8), [1.5 + 0.1j], 0.0)
    ctx.set_target(synth.sphere_occupancy(8), [1.5 + 0.1j], 0.3)
    kh, es, _ = dda.waves_for_orientation(0.1, 0.2, 0.3)
    _, st, _ = ctx.solve([kh, kh], es, want_p=False)
    assert all(s["rel_resid"] <= 1e-5 for s in st)


def test_rejected_solves(ctx):
    import paper_1002_1505_amd as P
    from paper_1002_1505_amd import _lib as L

    ctx.set_target(synth.sphere_occupancy(8), [1.5 + 0.1j], 0.3)
    kh, es, _ = dda.waves_for_orientation(0.0, 0.0, 0.0)
    with pytest.raises(P.DDAError):  # |khat| != 1
        ctx.solve([2 * kh], es[:1], want_p=False)
    with pytest.raises(P.DDAError):  # unknown target id
        ctx.solve([kh], es[:1], targets=[3], want_p=False)
    with pytest.raises(P.DDAError):  # unknown guess kind
        ctx.solve([kh], es[:1], guess=9, want_p=False)
    opts = L.dda_solve_opts(tol=1e-5, max_iter=100, guess=0, prec=P.DDA_SOLVE_FP32_REFINE)
    w = (L.dda_wave * 1)()
    assert ctx.lib.dda_solve(ctx.h, 0, w, C.byref(opts), None, None, None) < 0  # no right-hand side
    _, st, _ = ctx.solve([kh], es[:1], want_p=False)
    assert st[0]["rel_resid"] <= 1e-5


def test_one_site_box_is_an_isolated_dipole(ctx):
    """2 x 2 x 2 box with one occupied site: P = alpha E exactly (no
    interaction term), for both precision modes."""
    import paper_1002_1505_amd as P

    occ = np.zeros((2, 2, 2), np.uint8)
    occ[1, 0, 1] = 1
    m, kd = 1.7 + 0.2j, 0.5
    ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
    kh, es, _ = dda.waves_for_orientation(0.3, 0.8, 1.2)
    r, comp, _ = dda.sites_from_occupancy(occ)
    for prec in (P.DDA_SOLVE_FP64, P.DDA_SOLVE_FP32_REFINE):
        Pg, st, _ = ctx.solve([kh, kh], es, prec=prec, tol=1e-10)
        for l in range(2):
            ainv = dda.site_inverse_polarizability(comp, [m], kd, dda.ALPHA_LDR, kh, es[l])
            ref = dda.incident_field(r, kd, kh, es[l]) / ainv[:, None]
            assert np.allclose(Pg[l], ref, rtol=1e-9, atol=0), (prec, l)


@pytest.mark.parametrize("n", [32, 64])
def test_wide_batch_matvec_vs_oracle(ctx, n):
    """12 right-hand sides in one matvec (more than one z-pass rhs group, all
    rhs of a tile on one XCD for n = 64), sampled rows against the oracle."""
    import paper_1002_1505_amd as P

    occ = synth.ellipsoid_occupancy((n, n, n), (n - 1.0, 0.8 * n, 0.6 * n))
    r, comp, _ = dda.sites_from_occupancy(occ)
    kd = 0.3
    ctx.set_target(occ, [1.4 + 0.05j], kd, P.DDA_ALPHA_LDR)
    rng = np.random.default_rng(n + 7)
    nr = 12
    x = rng.standard_normal((nr, len(r), 3)) + 1j * rng.standard_normal((nr, len(r), 3))
    ainv = (1.5 + 0.1 * np.arange(nr) + 0.2j)[:, None]
    rows = rng.choice(len(r), 24, replace=False)
    for prec, tol in ((P.DDA_FP32, 5e-6), (P.DDA_FP64, 1e-12)):
        y = ctx.matvec(x, ainv=ainv, prec=prec)
        for s in range(nr):
            ref = dda.matvec_rows(r, kd, np.full(len(r), ainv[s, 0]), x[s], rows)
            err = np.linalg.norm(y[s][rows] - ref) / np.linalg.norm(ref)
            assert err < tol, (n, prec, s, err)
