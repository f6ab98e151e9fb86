"""COCG (oracle/dda.py cocg) for the complex symmetric DDA matrix: the
solution against the dense LU solve, the bilinear orthogonality of its
residuals (r_i^T r_j = 0 for i != j, the property that defines the method),
and the matvec counts of COCG and BiCGstab on seeded small targets (one
matvec per COCG iteration against two per BiCGstab iteration)."""
import numpy as np
import pytest

import synth
from oracle import dda


def _system(seed, shape=(7, 6, 5), m=1.5 + 0.05j, k=0.5):
    rng = np.random.default_rng(seed)
    occ = synth.ellipsoid_occupancy(shape, tuple(0.95 * s for s in shape))
    r, comp, _ = dda.sites_from_occupancy(occ)
    kh, es, _ = dda.waves_for_orientation(*rng.uniform(0, 1.5, 3))
    ainv = dda.site_inverse_polarizability(comp, [m], k, dda.ALPHA_LDR, kh, es[0])
    E = dda.incident_field(r, k, kh, es[0])
    return r, k, ainv, E


def test_matrix_is_complex_symmetric():
    r, k, ainv, E = _system(0)
    A = dda.dense_matrix(r, k, ainv)
    assert np.allclose(A, A.T, rtol=0, atol=1e-13 * np.abs(A).max())


@pytest.mark.parametrize("seed", range(3))
def test_cocg_solves_the_dense_system(seed):
    r, k, ainv, E = _system(seed)
    A = dda.dense_matrix(r, k, ainv)
    x, info = dda.cocg(lambda v: A @ v, E.reshape(-1), tol=1e-12)
    want = dda.solve_dense(r, k, ainv, E).reshape(-1)
    assert info["rel_resid"] <= 1e-12
    assert np.linalg.norm(x - want) / np.linalg.norm(want) < 1e-10


def test_cocg_residuals_are_bilinear_orthogonal():
    r, k, ainv, E = _system(4, shape=(5, 4, 4))
    A = dda.dense_matrix(r, k, ainv)
    _, info = dda.cocg(lambda v: A @ v, E.reshape(-1), tol=1e-9, keep_residuals=True)
    R = np.array(info["residuals"][:8])
    G = R @ R.T  # bilinear, no conjugation
    d = np.abs(np.diag(G))
    off = np.abs(G - np.diag(np.diag(G))) / np.sqrt(d[:, None] * d[None, :])
    assert off.max() < 1e-8


@pytest.mark.parametrize("m,k", [(1.5 + 0.05j, 0.5), (1.33 + 0.01j, 0.45), (1.7 + 0.2j, 0.4)])
def test_cocg_and_bicgstab_matvec_counts(m, k):
    """Both reach 1e-5; COCG's matvec count stays within a factor 1.5 of
    BiCGstab's on these targets (the two methods cost about the same per
    matvec)."""
    r, k, ainv, E = _system(7, shape=(8, 7, 6), m=m, k=k)
    mv = lambda v: dda.matvec_direct(r, k, ainv, v.reshape(-1, 3)).reshape(-1)
    _, ic = dda.cocg(mv, E.reshape(-1), tol=1e-5)
    _, ib = dda.bicgstab(mv, E.reshape(-1), tol=1e-5)
    assert ic["rel_resid"] <= 1e-5 and ib["rel_resid"] <= 1e-5
    assert ic["matvecs"] <= 1.5 * ib["matvecs"] and ib["matvecs"] <= 1.5 * ic["matvecs"], (ic, ib)


def _small_system(seed, m=1.7 + 0.02j, kd=0.5):
    occ = synth.ellipsoid_occupancy((10, 12, 8), (9.5, 11.5, 7.5))
    r, comp, _ = dda.sites_from_occupancy(occ)
    kh, es, _ = dda.waves_for_orientation(0.3 + seed, 0.8, 0.1)
    ainv = dda.site_inverse_polarizability(comp, [m], kd, dda.ALPHA_LDR, kh, es[0])
    E = dda.incident_field(r, kd, kh, es[0]).reshape(-1)
    A = dda.dense_matrix(r, kd, ainv)
    return A, E


def test_bicgstab_ell_one_is_bicgstab():
    """BiCGstab(1) takes the same iterates as BiCGstab (two independent codes
    of the same recurrences), cycle by cycle."""
    A, E = _small_system(0)
    mv = lambda v: A @ v
    for k in (1, 2, 5, 10):
        x1, _ = dda.bicgstab_l(mv, E, ell=1, tol=0, max_iter=k)
        x2, _ = dda.bicgstab(mv, E, tol=0, max_iter=k)
        assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x2), k


@pytest.mark.parametrize("ell", [1, 2, 4])
def test_bicgstab_ell_solves_the_dense_system(ell):
    """BiCGstab(ell) reaches the LU solution; its recursive residual r_0 is
    the residual of its iterate (the true residual agrees at the end); the
    iteration count is a multiple of ell (convergence is checked at the end
    of a cycle)."""
    A, E = _small_system(1)
    Pd = np.linalg.solve(A, E)
    x, info = dda.bicgstab_l(lambda v: A @ v, E, ell=ell, tol=1e-10, keep_residuals=True)
    assert info["rel_resid"] <= 1e-10 * 1.01
    assert np.linalg.norm(x - Pd) <= 1e-8 * np.linalg.norm(Pd)
    assert abs(info["residuals"][-1] - info["rel_resid"]) <= 1e-12
    assert info["iters"] % ell == 0 and info["matvecs"] == 2 * info["iters"] + 2  # + initial and final residual
