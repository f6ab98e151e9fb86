"""dda_matvec_noalloc, the matvec entry point that allocates nothing (its
intermediates live in the library's fixed per-GPU scratch array), against
dda_matvec, the entry point that allocates its workspaces: two calls in a
row, the second with a smaller input, in both precisions, plus its error
paths (spectrum not built, scratch need above the limit)."""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle import dda

pytestmark = pytest.mark.gpu


class _Dev:
    """Device memory and copies from the HIP runtime the library itself uses
    (its soname, so the process has one runtime); the test allocates its own
    inputs and outputs, the entry point under test allocates nothing."""

    def __init__(self):
        from paper_1002_1505_amd import _lib as L

        L.load()
        self.hip = C.CDLL("libamdhip64.so.7")
        self.live = []

    def put(self, a):
        a = np.ascontiguousarray(a)
        p = C.c_void_p()
        assert self.hip.hipMalloc(C.byref(p), C.c_size_t(a.nbytes)) == 0
        assert self.hip.hipMemcpy(p, C.c_void_p(a.ctypes.data), C.c_size_t(a.nbytes), 1) == 0  # host to device
        self.live.append(p)
        return p

    def get(self, p, like):
        out = np.empty_like(like)
        assert self.hip.hipDeviceSynchronize() == 0  # the context's stream does not order with hipMemcpy
        assert self.hip.hipMemcpy(C.c_void_p(out.ctypes.data), p, C.c_size_t(out.nbytes), 2) == 0  # to host
        return out

    def free(self):
        for p in self.live:
            self.hip.hipFree(p)
        self.live = []


def _noalloc(ctx, dev, target, x, ainv, prec):
    import paper_1002_1505_amd as P

    x = np.ascontiguousarray(x, dtype=np.complex128)
    xd = dev.put(x)
    yd = dev.put(np.full_like(x, complex(np.nan, np.nan)))  # every output element must be written
    ad = dev.put(np.ascontiguousarray(ainv, dtype=np.complex128))
    st = ctx.lib.dda_matvec_noalloc(ctx.h, int(target), x.shape[0], ad, xd, yd, int(prec))
    if st < 0:
        dev.free()
        raise P.DDAError(st, ctx.last_error())
    y = dev.get(yd, x)
    dev.free()
    return y


def test_noalloc_matvec_matches_dda_matvec():
    import paper_1002_1505_amd as P

    dev = _Dev()
    with P.Context(0) as ctx:
        occs = [synth.sphere_occupancy(32), synth.ellipsoid_occupancy((20, 24, 18), (19.0, 23.0, 17.5))]
        ctx.set_target(occs[0], [1.5 + 0.1j], 0.4, P.DDA_ALPHA_LDR)
        ctx.add_target(occs[1], [1.33 + 0.01j, 1.7 + 0.2j], 0.3, P.DDA_ALPHA_LDR)
        ctx.build_green_fft(P.DDA_FP32 | P.DDA_FP64)
        rng = np.random.default_rng(17)
        for prec, tol in ((P.DDA_FP64, 1e-13), (P.DDA_FP32, 1e-6)):
            # two calls in a row, the second with a smaller input (fewer rhs, smaller target)
            for target, nrhs in ((0, 3), (1, 1)):
                n = ctx.n_sites[target]
                ncomp = 1 if target == 0 else 2
                x = rng.standard_normal((nrhs, n, 3)) + 1j * rng.standard_normal((nrhs, n, 3))
                ainv = (rng.standard_normal((nrhs, ncomp)) + 1j * rng.standard_normal((nrhs, ncomp))) + 2.0
                print(f"noalloc prec={prec} target={target} nrhs={nrhs} N={n}", flush=True)
                ref = ctx.matvec(x, target=target, ainv=ainv, prec=prec)
                y = _noalloc(ctx, dev, target, x, ainv, prec)
                assert np.all(np.isfinite(y))
                err = np.abs(y - ref).max() / np.abs(ref).max()
                print(f"  max rel diff {err:.3e} bit-identical {np.array_equal(y, ref)}", flush=True)
                assert err <= tol
        # 4 FP32 rhs of a 64^3 box need about 127 MB of scratch: rejected
        ctx.set_target(synth.sphere_occupancy(64), [1.5 + 0.1j], 0.3, P.DDA_ALPHA_LDR)
        n = ctx.n_sites[0]
        x = np.zeros((4, n, 3), np.complex128)
        with pytest.raises(P.DDAError) as ei:  # spectrum not built yet
            _noalloc(ctx, dev, 0, x, np.ones((4, 1)), P.DDA_FP32)
        assert ei.value.status == -4
        ctx.build_green_fft(P.DDA_FP32)
        with pytest.raises(P.DDAError) as ei:
            _noalloc(ctx, dev, 0, x, np.ones((4, 1)), P.DDA_FP32)
        assert ei.value.status == -1 and "limit" in str(ei.value)
        # 2 FP32 rhs of the 64^3 box fit
        x = rng.standard_normal((2, n, 3)) + 1j * rng.standard_normal((2, n, 3))
        ainv = np.full((2, 1), dda.inverse_polarizability(1.5 + 0.1j, 0.3, dda.ALPHA_CM))
        y = _noalloc(ctx, dev, 0, x, ainv, P.DDA_FP32)
        ref = ctx.matvec(x, ainv=ainv, prec=P.DDA_FP32)
        assert np.abs(y - ref).max() / np.abs(ref).max() <= 1e-6
