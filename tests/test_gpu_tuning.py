"""Every launch shape the autotuner can pick computes the same product, and
the tuner's cache round-trips.  Expected values from the oracle's direct sum."""
import json
import os

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


def _shapes():
    out = []
    for tx in (8, 16, 32):
        for zrb in (0, 1, 2, 3):
            for ct in (3, 7, 11, 15):  # 8: class-grouped slab (n = 64, z pass variant 3)
                out.append(dict(fused=1, nth_plane=256, nth_z=256, tx=tx, lines_tl=16, nth_lines=256, ct=ct, zrb=zrb))
    for tx in (4, 8, 16):
        for fused in (1, 0):
            out.append(dict(fused=fused, nth_plane=256, nth_z=512, tx=tx, lines_tl=16, nth_lines=256, ct=0, zrb=0))
    return out


@pytest.mark.parametrize("n", [16, 32, 48, 64])
def test_all_launch_shapes_agree_with_oracle(ctx, n):
    import paper_1002_1505_amd as P

    occ = synth.sphere_occupancy(n)
    r, comp, _ = dda.sites_from_occupancy(occ)
    kd = 0.35
    ctx.set_target(occ, [1.5 + 0.1j], kd, P.DDA_ALPHA_LDR)
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, len(r), 3)) + 1j * rng.standard_normal((3, len(r), 3))
    ainv = np.array([[2.0 + 0.3j], [1.0 - 0.2j], [3.0 + 0.0j]])
    rows = rng.choice(len(r), 40, replace=False)
    refs = [dda.matvec_rows(r, kd, np.full(len(r), ainv[s, 0]), x[s], rows) for s in range(3)]
    tried = 0
    for prec, tol in ((P.DDA_FP32, 5e-6), (P.DDA_FP64, 1e-12)):
        for sh in _shapes():
            try:
                ctx.set_shape(sh, prec=prec)
            except P.DDAError:
                continue  # does not fit LDS / threads for this box
            tried += 1
            y = ctx.matvec(x, ainv=ainv, prec=prec)
            for s in range(3):
                err = np.sqrt(np.mean(np.abs(y[s][rows] - refs[s]) ** 2)) / np.sqrt(np.mean(np.abs(refs[s]) ** 2))
                assert err < tol, (n, prec, sh, err)
    assert tried >= 8


def test_autotune_cache_roundtrip(ctx, tmp_path):
    import paper_1002_1505_amd as P

    occ = synth.sphere_occupancy(32)
    ctx.set_target(occ, [1.4 + 0.05j], 0.3)
    path = str(tmp_path / "tune.json")
    ctx.autotune(2, path)
    s32, s64 = ctx.get_shape(prec=P.DDA_FP32), ctx.get_shape(prec=P.DDA_FP64)
    data = json.load(open(path))
    assert len(data) == 2
    # a new context reads the cache instead of timing, and picks the same shapes
    with P.Context(0) as c2:
        c2.set_target(occ, [1.4 + 0.05j], 0.3)
        c2.autotune(2, path)
        assert c2.get_shape(prec=P.DDA_FP32) == s32 and c2.get_shape(prec=P.DDA_FP64) == s64
    assert os.path.getsize(path) > 0
    # the tuned shape still solves correctly
    khat, e0 = P.orientation_waves(0.2, 0.3, 0.4)
    Pg, st, status = ctx.solve(khat, e0)
    assert status == 0 and all(s["rel_resid"] <= 1e-5 for s in st)


def test_two_factor_zpass_128_matches_lds_zpass_and_oracle(ctx):
    """The 128^3 box's FP32 two-factor z pass (variant 4: 16 x 8, one
    frequency parity per block half, the 16-point step split over lane pairs),
    in the row slab layout and in the class-grouped layout (Hadamard of the
    quadrant partners in the z pass, one load per frequency in the inverse
    pass), against the LDS-line z pass (variant 1) on the full vectors,
    element by element, and against the oracle's direct sum on sampled rows."""
    import paper_1002_1505_amd as P

    occ = synth.sphere_occupancy(128)
    r, comp, _ = dda.sites_from_occupancy(occ)
    kd = 0.3124
    ctx.set_target(occ, [1.33 + 0.01j], kd, P.DDA_ALPHA_LDR)
    sh = ctx.get_shape(prec=P.DDA_FP32)
    assert sh["zrb"] == 4 and sh["tx"] == 8, sh
    rng = np.random.default_rng(128)
    x = rng.standard_normal((2, len(r), 3)) + 1j * rng.standard_normal((2, len(r), 3))
    ainv = np.array([[2.0 + 0.3j], [1.0 - 0.2j]])
    ys = {}
    for name, shp in (("row", dict(sh, ct=sh["ct"] & ~8)), ("grouped", dict(sh, ct=sh["ct"] | 8)),
                      ("lines", dict(sh, ct=sh["ct"] & ~8, zrb=1, tx=8))):
        ctx.set_shape(shp, prec=P.DDA_FP32)
        ys[name] = ctx.matvec(x, ainv=ainv, prec=P.DDA_FP32)
    ctx.set_shape(sh, prec=P.DDA_FP32)
    rows = np.concatenate([[0, len(r) - 1], rng.choice(len(r), 30, replace=False)])
    y1 = ys["lines"]
    for name in ("row", "grouped"):
        y4 = ys[name]
        for s in range(2):
            d = np.abs(y4[s] - y1[s])
            scale = np.sqrt(np.mean(np.abs(y1[s]) ** 2))
            print(f"{name} rhs {s}: rms diff {np.sqrt(np.mean(d ** 2)) / scale:.2e}, max diff {d.max() / scale:.2e}",
                  flush=True)
            assert np.sqrt(np.mean(d ** 2)) / scale < 2e-6 and d.max() / scale < 2e-5
            ref = dda.matvec_rows(r, kd, np.full(len(r), ainv[s, 0]), x[s], rows)
            err = np.abs(y4[s][rows] - ref).max() / np.sqrt(np.mean(np.abs(ref) ** 2))
            assert err < 2e-5, err
