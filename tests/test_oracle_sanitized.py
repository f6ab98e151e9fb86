"""The oracle's C direct sum built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only, any report is fatal) and run
on seeded inputs, including the one-site and empty row-sample cases: no
report, and the same products as the regular OpenMP build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import dda

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_C = os.path.join(os.path.dirname(HERE), "oracle", "direct.c")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    d = tmp_path_factory.mktemp("asan")
    exe = str(d / "direct_asan")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", ORACLE_C,
           os.path.join(HERE, "sanitize", "direct_driver.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True)
    return exe, d


def _run(driver, r, k, ainv, x, rows):
    exe, d = driver
    inp, out = str(d / "in.bin"), str(d / "out.bin")
    n = len(r)
    with open(inp, "wb") as f:
        np.array([n, len(rows)], dtype=np.int64).tofile(f)
        np.array([k], dtype=np.float64).tofile(f)
        np.ascontiguousarray(r, dtype=np.float64).tofile(f)
        np.ascontiguousarray(ainv, dtype=np.complex128).tofile(f)
        np.ascontiguousarray(x, dtype=np.complex128).tofile(f)
        np.ascontiguousarray(rows, dtype=np.int64).tofile(f)
    env = dict(os.environ, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    p = subprocess.run([exe, inp, out], env=env, capture_output=True, text=True)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-4000:]
    raw = np.fromfile(out, dtype=np.complex128)
    return raw[: 3 * n].reshape(n, 3), raw[3 * n:].reshape(len(rows), 3)


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 1, 1), (5, 4, 3), (9, 7, 6)])
def test_direct_sum_clean_under_sanitizers(driver, shape):
    rng = np.random.default_rng(sum(shape))
    occ = np.ones(shape, dtype=bool)
    if occ.size > 4:
        occ &= rng.random(shape) < 0.8
        occ.flat[0] = True
    r, comp, _ = dda.sites_from_occupancy(occ)
    n = len(r)
    k = 0.37
    ainv = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    rows = rng.choice(n, min(n, 7), replace=False).astype(np.int64)
    y, ys = _run(driver, r, k, ainv, x, rows)
    ref = dda.matvec_direct(r, k, ainv, x)
    assert np.allclose(y, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    assert np.allclose(ys, ref[rows], rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    # no rows sampled: the row product writes nothing and reads nothing
    y0, ys0 = _run(driver, r, k, ainv, x, np.zeros(0, dtype=np.int64))
    assert ys0.shape == (0, 3) and np.array_equal(y0, y)
