"""dda_near_field on the GPU: E and B at points against the oracle's dipole
sums from its own dense solution, and, at the bench size, the DDA's local-
field identity (the field at an occupied site is 1/alpha P) on sampled
sites."""
import numpy as np
import pytest

import synth
from oracle import dda, nearfield

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1002_1505_amd as P

    c = P.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("kind", [dda.ALPHA_CM, dda.ALPHA_LDR])
def test_near_field_vs_oracle(ctx, kind):
    import paper_1002_1505_amd as P

    occ = synth.ellipsoid_occupancy((8, 6, 5), (7.6, 5.5, 4.6))
    r, comp, _ = dda.sites_from_occupancy(occ)
    k, m = 0.5, 1.6 + 0.2j
    kinds = {dda.ALPHA_CM: P.DDA_ALPHA_CM, dda.ALPHA_LDR: P.DDA_ALPHA_LDR}
    ctx.set_target(occ, [m], k, kinds[kind])
    kh, es, L = dda.waves_for_orientation(0.4, 1.0, 0.3)
    _, st, _ = ctx.solve([kh, kh], es, prec=P.DDA_SOLVE_FP64, tol=1e-12, want_p=False)
    assert all(s["rel_resid"] <= 1e-12 for s in st)
    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 29)
    pts = np.concatenate([
        rng.uniform(-6, 6, size=(24, 3)),                               # in and around the target
        r[rng.choice(len(r), size=6, replace=False)],                   # on occupied sites
        np.linspace([-12.0, 0.3, -0.2], [12.0, 0.3, -0.2], 25),          # a track through it
        np.array([[0.0, 0.0, 40.0], [300.0, -200.0, 150.0]]),           # farther out
    ])
    E, B = ctx.near_field(2, pts)
    for l in range(2):
        ainv = dda.site_inverse_polarizability(comp, [m], k, kind, kh, es[l])
        Pw = dda.solve_dense(r, k, ainv, dda.incident_field(r, k, kh, es[l]))
        Eo, Bo = nearfield.near_field(r, Pw, k, kh, es[l], pts)
        assert _rel(E[l], Eo) < 1e-9, l
        assert _rel(B[l], Bo) < 1e-9, l
        for q in range(len(pts)):  # every point, not only the norm
            assert np.linalg.norm(E[l][q] - Eo[q]) <= 1e-8 * np.linalg.norm(Eo[q]) + 1e-12, (l, q)


def test_local_field_identity_at_bench_size(ctx):
    """Sphere in the 64^3 box (N = 137,376), FP32 matvec with FP64
    refinement to 1e-5: the field at sampled occupied sites is 1/alpha P to
    the solve's residual."""
    import paper_1002_1505_amd as P

    occ = synth.sphere_occupancy(64)
    r, comp, _ = dda.sites_from_occupancy(occ)
    kd = 10.0 / dda.effective_radius(len(r))
    ctx.set_target(occ, [1.5 + 0.1j], kd, P.DDA_ALPHA_LDR)
    kh, e0 = P.orientation_waves(0.0, 0.0, 0.0)
    Pl, st, _ = ctx.solve(list(kh), list(e0), tol=1e-5)
    assert all(s["rel_resid"] <= 1e-5 for s in st)
    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 31)
    sel = rng.choice(len(r), size=64, replace=False)
    E, B = ctx.near_field(2, r[sel], want_b=False)
    assert B is None
    for l in range(2):
        a = ctx.inverse_polarizability(kh[l], e0[l])  # (Re, Im) per composition
        want = (a[0] + 1j * a[1]) * Pl[l][sel]
        assert _rel(E[l], want) < 1e-4, l


def test_two_targets_in_one_call(ctx):
    """A solve over two targets (one rhs each) with caller fields, then the
    near field of both: each rhs equals the single-target call, each target
    in its own frame (origin at its own centroid)."""
    import paper_1002_1505_amd as P

    occs = [synth.ellipsoid_occupancy((8, 6, 5), (7.6, 5.5, 4.6)), synth.sphere_occupancy(8)]
    ms, ks = [1.6 + 0.2j, 1.4 + 0.05j], [0.5, 0.4]
    kh, es, L = dda.waves_for_orientation(0.2, 0.7, 1.1)
    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 37)
    sites = [dda.sites_from_occupancy(o)[0] for o in occs]
    E = [rng.standard_normal((len(r), 3)) + 1j * rng.standard_normal((len(r), 3)) for r in sites]
    pts = rng.uniform(-7, 7, size=(12, 3))
    ctx.set_target(occs[0], [ms[0]], ks[0], P.DDA_ALPHA_LDR)
    ctx.add_target(occs[1], [ms[1]], ks[1], P.DDA_ALPHA_LDR)
    Pb, sb, _ = ctx.solve([kh, kh], [es[0], es[1]], targets=[0, 1], prec=P.DDA_SOLVE_FP64, tol=1e-11, e_inc=E)
    Eb, Bb = ctx.near_field(2, pts)
    for t in range(2):
        ctx.set_target(occs[t], [ms[t]], ks[t], P.DDA_ALPHA_LDR)
        Ps, ss, _ = ctx.solve([kh], [es[t]], prec=P.DDA_SOLVE_FP64, tol=1e-11, e_inc=[E[t]])
        Es, Bs = ctx.near_field(1, pts)
        assert _rel(Pb[t], Ps[0]) < 1e-9, t
        assert _rel(Eb[t], Es[0]) < 1e-9 and _rel(Bb[t], Bs[0]) < 1e-9, t


def test_near_field_errors():
    import ctypes as C

    import paper_1002_1505_amd as P
    from paper_1002_1505_amd import _lib as L

    c = P.Context(0)
    try:
        c.set_target(synth.sphere_occupancy(6), [1.5 + 0.1j], 0.4)
        E = np.zeros(12)
        pts = np.zeros(3)
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        assert c.lib.dda_near_field(c.h, 1, 1, dp(pts), dp(E), None) == L.DDA_ERR_STATE  # before a solve
        kh, e0 = P.orientation_waves(0.0, 0.0, 0.0)
        c.solve(list(kh), list(e0), tol=1e-6, want_p=False)
        assert c.lib.dda_near_field(c.h, 1, 1, dp(pts), dp(E), None) == L.DDA_ERR_INVALID_ARG  # 2 rhs solved
        assert c.lib.dda_near_field(c.h, 2, 0, dp(pts), dp(E), None) == L.DDA_ERR_INVALID_ARG
        assert c.lib.dda_near_field(c.h, 2, 1, None, dp(E), None) == L.DDA_ERR_INVALID_ARG
        with pytest.raises(P.DDAError):
            c.near_field(1, [[0.0, 0.0, 5.0]])
    finally:
        c.close()
