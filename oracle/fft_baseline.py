"""CPU timing baseline of the FFT method (test infrastructure only; not the
parity oracle).

It applies the same operator as ``dda.matvec_direct`` through the convolution
theorem. The off-diagonal blocks A(r_j - r_l) depend only on the lattice
separation, so the interaction part of A P is a three-component discrete
convolution of the site polarizations with the interaction tensor. It is
evaluated on a zero-padded grid at least twice the target's extent per axis,
which is the guide's FFT approach to the matvec (section "Choice of FFT
Algorithm"). The host FFTs are numpy/scipy; the diagonal 1/alpha term is
added per site.

Its purpose is to time the FFT algorithm on the host cores beside the GPU
library. Its agreement with the direct pair sum (exact up to FFT rounding)
is pinned in tests. It shares no code with the GPU library.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import dda


class FftDda:
    """A x = sum_l A(r_j - r_l) x_l + (1/alpha_j) x_j for the sites r (N, 3)
    of one target, in complex128 or complex64 arithmetic."""

    def __init__(self, r, k, ainv, dtype=np.complex128, workers=-1):
        r = np.asarray(r, dtype=np.float64)
        self.idx = np.rint(r - r.min(axis=0)).astype(np.int64)  # lattice indices (x, y, z) from 0
        ext = self.idx.max(axis=0) + 1
        # no wrap-around: every separation fits in (-M/2, M/2)
        self.M = tuple(int(sfft.next_fast_len(int(2 * e))) for e in ext)
        self.dtype = np.dtype(dtype)
        self.workers = workers
        self.ainv = np.broadcast_to(np.asarray(ainv, dtype=np.complex128), (len(r),)).astype(self.dtype)
        self.ghat = self._tensor_spectrum(k, ext)

    def _tensor_spectrum(self, k, ext):
        # separation d along each axis at grid index i: i, or i - M past the middle
        lag = []
        for M, e in zip(self.M, ext):
            i = np.arange(M)
            d = np.where(i < M // 2, i, i - M).astype(np.float64)
            d[np.abs(d) >= e] = np.nan  # separations no pair of sites has
            lag.append(d)
        dx, dy, dz = np.meshgrid(lag[0], lag[1], lag[2], indexing="ij")
        rr = np.sqrt(dx * dx + dy * dy + dz * dz)
        valid = np.isfinite(rr) & (rr > 0)
        rs = np.where(valid, rr, 1.0)
        n = [np.where(valid, d / rs, 0.0) for d in (dx, dy, dz)]
        ph = np.where(valid, np.exp(1j * k * rs) / rs, 0.0)
        c1 = k * k
        c2 = (1j * k * rs - 1.0) / rs ** 2
        ghat = {}
        for a in range(3):
            for b in range(a, 3):
                nn = n[a] * n[b]
                delta = 1.0 if a == b else 0.0
                g = ph * (c1 * (nn - delta) + c2 * (3.0 * nn - delta))
                ghat[(a, b)] = sfft.fftn(g, workers=self.workers).astype(self.dtype)
        return ghat

    def matvec(self, x):
        x = np.asarray(x).reshape(-1, 3).astype(self.dtype)
        ix, iy, iz = self.idx[:, 0], self.idx[:, 1], self.idx[:, 2]
        X = []
        for c in range(3):
            g = np.zeros(self.M, dtype=self.dtype)
            g[ix, iy, iz] = x[:, c]
            X.append(sfft.fftn(g, workers=self.workers))
        y = np.empty_like(x)
        for a in range(3):
            Y = sum(self.ghat[(min(a, b), max(a, b))] * X[b] for b in range(3))
            y[:, a] = sfft.ifftn(Y, workers=self.workers)[ix, iy, iz]
        return y + self.ainv[:, None] * x

    def solve(self, E, tol=1e-5, max_iter=10000):
        """BiCGstab (the oracle's) over this matvec; E, P are (N, 3)."""
        n = len(self.idx)
        mv = lambda v: self.matvec(v.reshape(n, 3)).reshape(-1).astype(np.complex128)
        P, info = dda.bicgstab(mv, np.asarray(E).reshape(-1), tol=tol, max_iter=max_iter)
        return P.reshape(n, 3), info
