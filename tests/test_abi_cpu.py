"""CPU-side checks of the C ABI: the built library loads and exports every
symbol that include/dda.h declares, and the Python binding declares them all.
No compute call is made (no GPU here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dda.h")
LIB = os.path.join(ROOT, "paper_1002_1505_amd", "libdda.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dda_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_core_calls():
    names = declared_functions()
    for must in ["dda_create", "dda_set_target", "dda_build_green_fft", "dda_solve", "dda_cross_sections",
                 "dda_amplitudes", "dda_matvec"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdda.so not built")
def test_library_exports_every_declared_symbol():
    import ctypes

    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_1002_1505_amd import _lib

    assert sorted(_lib.SIGNATURES) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdda.so not built")
def test_host_only_calls_without_gpu():
    """dda_lab_frame and dda_mueller are host arithmetic; checked against the
    oracle's frame and Mueller formulas."""
    import numpy as np

    import paper_1002_1505_amd as P
    from oracle import dda, scatter

    for b, t, p in [(0.1, 0.2, 0.3), (2.0, 1.0, -0.5)]:
        assert np.allclose(P.lab_frame(b, t, p), dda.lab_axes_in_target_frame(b, t, p), atol=1e-14)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((5, 2, 2)) + 1j * rng.standard_normal((5, 2, 2))
    phi = rng.uniform(0, 6, 5)
    e01, e02 = dda.incident_polarizations((0, 1, 0.5j))
    S, M = P.mueller(f, phi, e01, e02)
    So = scatter.amplitude_matrix(f, phi, e01, e02)
    assert np.allclose(S, So, atol=1e-13)
    assert np.allclose(M, scatter.mueller(So), atol=1e-12)


def test_no_device_error_is_clean():
    """Creating a context without a GPU returns an error, it does not crash."""
    import paper_1002_1505_amd as P

    if not os.path.exists(LIB):
        pytest.skip("libdda.so not built")
    try:
        import torch

        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except Exception:
        pass
    with pytest.raises(P.DDAError):
        P.Context(0)


def test_orientation_helpers_without_gpu():
    """dda_orientation_samples and dda_phi_coefficients are host arithmetic;
    checked against the oracle's sampling rules and polarization projection."""
    import numpy as np

    import paper_1002_1505_amd as P
    from oracle import orient as O

    lims = np.deg2rad([0, 360, 0, 180, 0, 360])
    for counts in [(1, 1, 1), (2, 3, 2), (3, 4, 5), (4, 7, 3)]:
        got, want = P.orientation_samples(lims, counts), O.orientation_samples(lims, counts)
        for g, w in zip(got, want):
            assert np.allclose(g, w, atol=1e-14)
    lims = np.deg2rad([10, 80, 20, 150, 5, 95])
    got, want = P.orientation_samples(lims, (3, 2, 4)), O.orientation_samples(lims, (3, 2, 4))
    for g, w in zip(got, want):
        assert np.allclose(g, w, atol=1e-14)
    rng = np.random.default_rng(2)
    for _ in range(4):
        be, th, p0 = rng.uniform(0, 2 * np.pi, 3)
        phis = rng.uniform(0, 2 * np.pi, 3)
        c = P.phi_coefficients(be, th, p0, phis)
        for k, ph in enumerate(phis):
            assert np.allclose(c[k], O.phi_coefficients(be, th, p0, ph), atol=1e-13)
    with pytest.raises(P.DDAError):
        P.orientation_samples(lims, (0, 1, 1))


def test_scattering_quadrature_without_gpu():
    """dda_scattering_quadrature is host arithmetic: the guide's worked
    example (x = 6.187304, ETASCA = 0.5) uses NAVG = 2292 directions, and the
    directions and weights equal the oracle's."""
    import numpy as np

    import paper_1002_1505_amd as P
    from oracle import dda, scatter

    L = dda.lab_axes_in_target_frame(0.0, 0.0, 0.0)
    n, w = P.scattering_quadrature(6.187304, 0.5, L)
    assert len(w) == 2292
    for x, eta, ang in [(6.187304, 0.5, (0, 0, 0)), (1.0, 0.5, (0.3, 1.1, 2.0)), (10.0, 1.0, (2.0, 0.4, 0.7)),
                        (0.2, 0.25, (1.0, 2.0, 3.0))]:
        L = dda.lab_axes_in_target_frame(*ang)
        n, w = P.scattering_quadrature(x, eta, L)
        no, wo = scatter.quadrature_directions_tf(x, eta, L)
        assert n.shape == no.shape and np.allclose(n, no, atol=1e-13) and np.allclose(w, wo, rtol=1e-13)
        assert abs(w.sum() - 4 * np.pi) < 0.05
    with pytest.raises(P.DDAError):
        P.scattering_quadrature(-1.0, 0.5, L)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdda.so not built")
def test_polarization_without_gpu():
    """dda_polarization (host arithmetic) against the oracle's polarized cross
    sections and linear polarization, for random amplitude matrices and
    incident states; bad arguments are rejected."""
    import numpy as np

    import paper_1002_1505_amd as P
    from oracle import scatter

    rng = np.random.default_rng(11)
    S = rng.standard_normal((9, 4)) + 1j * rng.standard_normal((9, 4))
    M = scatter.mueller(S)
    k = 0.61
    for stokes in ([1, 0, 0, 0], [1, 1, 0, 0], [1, -1, 0, 0], [2.0, 0.4, -1.1, 0.9], [1, 0, 0, -1]):
        got = P.polarization(M, k, stokes)
        assert np.allclose(got[:, :3], scatter.polarized_cross_sections(M, k, stokes), rtol=1e-12, atol=1e-15)
        assert np.allclose(got[:, 3], scatter.linear_polarization(M), rtol=1e-12)
    for bad in (dict(k=0.0), dict(stokes_in=[0, 1, 0, 0])):
        with pytest.raises(P.DDAError):
            P.polarization(M, bad.get("k", k), bad.get("stokes_in", [1, 0, 0, 0]))
