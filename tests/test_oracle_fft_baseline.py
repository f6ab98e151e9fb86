"""The host FFT timing baseline (oracle/fft_baseline.py) against the oracle's
direct pair sum: the same operator through the convolution theorem, exact up
to FFT rounding, and its BiCGstab solve against the dense LU solve."""
import numpy as np
import pytest

import synth
from oracle import dda, fft_baseline

TARGETS = [
    ("ellipsoid_9x8x7", lambda: synth.ellipsoid_occupancy((9, 8, 7), (8.6, 7.5, 6.4))),
    ("sphere_12", lambda: synth.sphere_occupancy(12)),
    ("ragged_9x11x6", lambda: (np.random.default_rng(3).random((6, 11, 9)) < 0.5).astype(np.uint8)),
]


def _case(build, k=0.45, m=1.5 + 0.1j):
    r, comp, _ = dda.sites_from_occupancy(build())
    ainv = dda.site_inverse_polarizability(comp, [m], k, dda.ALPHA_LDR, np.array([1.0, 0, 0]),
                                           np.array([0, 1.0, 0]))
    return r, ainv, k


@pytest.mark.parametrize("name,build", TARGETS, ids=[t[0] for t in TARGETS])
def test_fft_matvec_equals_direct_pair_sum(name, build):
    r, ainv, k = _case(build)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((len(r), 3)) + 1j * rng.standard_normal((len(r), 3))
    want = dda.matvec_direct(r, k, ainv, x)
    for dtype, bar in ((np.complex128, 1e-13), (np.complex64, 3e-7)):
        got = fft_baseline.FftDda(r, k, ainv, dtype=dtype).matvec(x)
        assert np.linalg.norm(got - want) / np.linalg.norm(want) < bar, dtype


def test_fft_grid_has_no_wraparound():
    r, ainv, k = _case(TARGETS[2][1])
    F = fft_baseline.FftDda(r, k, ainv)
    ext = F.idx.max(axis=0) + 1
    assert all(M >= 2 * e - 1 for M, e in zip(F.M, ext))


def test_fft_solve_matches_dense_lu():
    r, ainv, k = _case(TARGETS[0][1])
    E = dda.incident_field(r, k, np.array([0.0, 0.6, 0.8]), np.array([1.0, 0.0, 0.0]))
    P, info = fft_baseline.FftDda(r, k, ainv).solve(E, tol=1e-11)
    want = dda.solve_dense(r, k, ainv, E)
    assert info["rel_resid"] <= 1e-11
    assert np.linalg.norm(P - want) / np.linalg.norm(want) < 1e-9
