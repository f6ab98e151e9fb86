"""Anisotropic compositions on the GPU (dda_set_anisotropic) against the
oracle's dense solve with per-site tensor polarizabilities (oracle/dda.py
anisotropic_inverse_polarizability, dense_matrix and cross_sections; pinned
in test_oracle_aniso.py): the matvec, FP64 and FP32-refined solves with
BiCGstab and BiCGstab(2) on a target that mixes an isotropic and a rotated
uniaxial composition, the isotropic limit, and the refused calls."""
import numpy as np
import pytest

import synth
from oracle import dda

pytestmark = pytest.mark.gpu

M_ISO = 1.45 + 0.03j
M3 = [1.62 + 0.05j, 1.35 + 0.02j, 1.35 + 0.02j]
ANG = (0.8, 0.5, -0.4)
KD = 0.42


@pytest.fixture(scope="module")
def ctx():
    import paper_1002_1505_amd as P

    c = P.Context(0)
    yield c
    c.close()


def _occ(shape=(12, 10, 8)):
    occ = synth.ellipsoid_occupancy(shape, tuple(s - 0.5 for s in shape))
    # composition 2 in the half x > centre
    half = np.zeros_like(occ)
    half[:, :, shape[0] // 2:] = 1
    return occ * (1 + half).astype(np.uint8) * (occ > 0)


def _site_tensors(comp, kh, e, m3=M3, ang=ANG, m_iso=M_ISO):
    T2 = dda.anisotropic_inverse_polarizability(m3, ang, KD, dda.ALPHA_LDR, kh, e)
    T1 = dda.inverse_polarizability(m_iso, KD, dda.ALPHA_LDR, kh, e) * np.eye(3)
    return np.stack([T1 if c == 1 else T2 for c in comp])


def _setup(ctx, occ):
    import paper_1002_1505_amd as P

    ctx.set_target(occ, [M_ISO, 1.5 + 0.0j], KD, P.DDA_ALPHA_LDR)
    assert ctx.set_anisotropic(2, M3, ANG) == 0
    r, comp, _ = dda.sites_from_occupancy(occ)
    assert set(np.unique(comp)) == {1, 2}
    return r, comp


def test_matvec_vs_oracle(ctx):
    import paper_1002_1505_amd as P

    occ = _occ()
    r, comp = _setup(ctx, occ)
    T = _site_tensors(comp, np.array([1.0, 0, 0]), np.array([0, 1.0, 0]))  # dda_matvec's wave
    A = dda.dense_matrix(r, KD, T)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, len(r), 3)) + 1j * rng.standard_normal((2, len(r), 3))
    for prec, tol in ((P.DDA_FP64, 1e-12), (P.DDA_FP32, 5e-6)):
        y = ctx.matvec(x, prec=prec)
        for s in range(2):
            ref = (A @ x[s].reshape(-1)).reshape(-1, 3)
            d = np.abs(y[s] - ref)
            assert np.linalg.norm(d) <= tol * np.linalg.norm(ref) and d.max() <= 10 * tol * np.abs(ref).max()


@pytest.mark.parametrize("solver", ["bicgstab", "bicgstab2"])
@pytest.mark.parametrize("prec_name", ["fp64", "fp32_refine"])
def test_solve_vs_oracle(ctx, solver, prec_name):
    import paper_1002_1505_amd as P

    occ = _occ()
    r, comp = _setup(ctx, occ)
    kh, es, _ = dda.waves_for_orientation(0.5, 1.2, 0.3)
    prec = P.DDA_SOLVE_FP64 if prec_name == "fp64" else P.DDA_SOLVE_FP32_REFINE
    sv = P.DDA_SOLVER_BICGSTAB if solver == "bicgstab" else P.DDA_SOLVER_BICGSTAB2
    Pg, st, status = ctx.solve([kh, kh], es, tol=1e-6, prec=prec, solver=sv)
    assert status == 0
    q = ctx.cross_sections(2)
    for l in range(2):
        T = _site_tensors(comp, kh, es[l])
        E = dda.incident_field(r, KD, kh, es[l])
        A = dda.dense_matrix(r, KD, T)
        res = E.reshape(-1) - A @ Pg[l].reshape(-1)
        rel = np.linalg.norm(res) / np.linalg.norm(E)
        assert rel <= 1e-6 and abs(rel - st[l]["rel_resid"]) <= 1e-9
        Po = np.linalg.solve(A, E.reshape(-1)).reshape(-1, 3)
        qo = np.array(dda.cross_sections(KD, E, Po, T))
        assert np.all(np.abs(q[l] - qo) <= 1e-4 * np.abs(qo)), (q[l], qo)
    # the anisotropic sites matter: the isotropic solve of the same target differs
    ctx.set_target(occ, [M_ISO, M3[1]], KD, P.DDA_ALPHA_LDR)
    Pi, _, _ = ctx.solve([kh, kh], es, tol=1e-6, prec=prec)
    assert np.linalg.norm(Pi[0] - Pg[0]) > 1e-3 * np.linalg.norm(Pg[0])


def test_equal_principal_indices_reproduce_isotropic(ctx):
    import paper_1002_1505_amd as P

    occ = _occ((10, 8, 8))
    kh, es, _ = dda.waves_for_orientation(0.2, 0.7, 1.1)
    ctx.set_target(occ, [M_ISO, 1.6 + 0.04j], KD, P.DDA_ALPHA_LDR)
    Pi, _, _ = ctx.solve([kh, kh], es, tol=1e-9, prec=P.DDA_SOLVE_FP64)
    qi = ctx.cross_sections(2)
    ctx.set_anisotropic(2, [1.6 + 0.04j] * 3, (1.1, -0.7, 2.3))
    Pa, _, _ = ctx.solve([kh, kh], es, tol=1e-9, prec=P.DDA_SOLVE_FP64)
    qa = ctx.cross_sections(2)
    for l in range(2):
        assert np.linalg.norm(Pa[l] - Pi[l]) <= 1e-8 * np.linalg.norm(Pi[l])
    assert np.allclose(qa, qi, rtol=1e-8)


def test_refused_calls(ctx):
    import paper_1002_1505_amd as P

    occ = _occ()
    _setup(ctx, occ)
    kh, es, _ = dda.waves_for_orientation(0.0, 0.4, 0.0)
    ctx.solve([kh, kh], es, want_p=False)
    for g in (P.DDA_GUESS_PREV_SHIFT, P.DDA_GUESS_PROJECT):
        with pytest.raises(P.DDAError):
            ctx.solve([kh, kh], es, guess=g, want_p=False)
    with pytest.raises(P.DDAError):
        ctx.cross_sections_phi(np.zeros((1, 1, 2, 2), np.complex128))
    with pytest.raises(P.DDAError):
        ctx.set_anisotropic(3, M3, ANG)  # no composition 3
    with pytest.raises(P.DDAError):
        ctx.set_anisotropic(1, [np.nan, 1.0, 1.0], ANG)
    # |m| k d >= 1 warns
    assert ctx.set_anisotropic(1, [3.0, 1.3, 1.3], ANG) == P.DDA_WARN_MKD_GE_1
