"""CPU oracle for the DDA hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct double-precision implementation of what the
GPU library computes: lattice sites, frames, incident field, polarizabilities,
the dense interaction matrix (LU solve), a direct O(N^2) matvec (C + OpenMP)
inside the oracle's own BiCGstab, cross sections, scattering amplitudes,
Mueller matrix, angular quadrature, orientation sampling and averaging, the
near field of the dipoles, and Mie theory for spheres.  ``fft_baseline`` is not part of the oracle proper:
it applies the same operator through host FFTs, only to time the FFT method
on the CPU beside the GPU (pinned to the direct matvec in tests).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (``paper_1002_1505_amd``)
never imports it, and it never imports the product.

Functions whose parity is unpinned (no test fixes them against the paper or
mathematics independent of the oracle): the numerical values of the LDR
coefficients b1, b2, b3 (recalled from Draine & Goodman 1993, not printed in
the guide), and the near field within d of a dipole, where the guide's
program applies a smoothing factor it does not print (``nearfield``).  Everything else is pinned by ``tests/test_oracle_*.py``.
"""
from . import dda, mie, nn, scatter  # noqa: F401
