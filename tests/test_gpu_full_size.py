"""GPU parity at the full workload sizes, checked on sampled outputs the
oracle computes one row at a time (direct O(N) sum per row), and through
properties that hold at any size.

 * sphere in a 64^3 box (N = 137,376), FFT grid 128^3, m = 1.5+0.1i, x = 10
 * sphere in a 128^3 box (N = 1,099,136), FFT grid 256^3, m = 1.33+0.01i, x = 20
   (its FP64 products use the global-memory plane fallback)
"""
import numpy as np
import pytest

import synth
from oracle import dda

pytestmark = pytest.mark.gpu

WORKLOADS = {
    "box64_grid128": dict(n=64, m=1.5 + 0.1j, x=10.0),
    "box128_grid256": dict(n=128, m=1.33 + 0.01j, x=20.0),
}


@pytest.fixture(scope="module")
def ctx():
    import paper_1002_1505_amd as P

    c = P.Context(0)
    yield c
    c.close()


def _problem(name):
    w = WORKLOADS[name]
    occ = synth.sphere_occupancy(w["n"])
    r, comp, _ = dda.sites_from_occupancy(occ)
    kd = w["x"] / dda.effective_radius(len(r))
    return occ, r, comp, kd, w["m"]


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_matvec_sampled_rows(ctx, name):
    import paper_1002_1505_amd as P

    occ, r, comp, kd, m = _problem(name)
    ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
    n = len(r)
    print(f"[{name}] N={n} kd={kd:.5f}", flush=True)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((1, n, 3)) + 1j * rng.standard_normal((1, n, 3))
    ainv = dda.inverse_polarizability(m, kd, dda.ALPHA_CM)
    rows = np.concatenate([[0, n - 1], rng.choice(n, 62, replace=False)])
    ref = dda.matvec_rows(r, kd, np.full(n, ainv), x[0], rows)
    scale = np.sqrt(np.mean(np.abs(ref) ** 2))
    for prec, tol in ((P.DDA_FP64, 1e-12), (P.DDA_FP32, 5e-6)):
        y = ctx.matvec(x, ainv=[[ainv]], prec=prec)[0]
        err = np.sqrt(np.mean(np.abs(y[rows] - ref) ** 2)) / scale
        print(f"[{name}] prec={prec} sampled rel err {err:.3e}", flush=True)
        assert err < tol


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_solve_sampled_residual_and_cross_sections(ctx, name):
    import paper_1002_1505_amd as P

    occ, r, comp, kd, m = _problem(name)
    ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
    n = len(r)
    khat, e0 = P.orientation_waves(0.4, 1.0, 0.3)
    Pg, st, status = ctx.solve(khat, e0, tol=1e-5, prec=P.DDA_SOLVE_FP32_REFINE)
    print(f"[{name}] stats {st}", flush=True)
    assert status == 0
    q = ctx.cross_sections(2)
    rng = np.random.default_rng(9)
    rows = rng.choice(n, 48, replace=False)
    for l in range(2):
        assert st[l]["rel_resid"] <= 1e-5
        ainv = dda.site_inverse_polarizability(comp, [m], kd, dda.ALPHA_LDR, khat[l], e0[l])
        E = dda.incident_field(r, kd, khat[l], e0[l])
        # residual at sampled sites, relative to the rms field: consistent with
        # a global relative residual <= 1e-5
        AP = dda.matvec_rows(r, kd, ainv, Pg[l], rows)
        rs = np.sqrt(np.mean(np.abs(E[rows] - AP) ** 2)) / np.sqrt(np.mean(np.abs(E) ** 2))
        print(f"[{name}] pol {l} sampled residual {rs:.2e}", flush=True)
        assert rs < 1e-4
        # the library's reductions on its own P equal the oracle's sums on that P
        qo = np.array(dda.cross_sections(kd, E, Pg[l], ainv))
        assert np.all(np.abs(q[l] - qo) / np.abs(qo) < 1e-9)
        assert q[l, 1] > 0 and q[l, 2] > 0
