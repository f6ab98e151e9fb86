"""Writes the stored oracle solutions that the full-size GPU tests compare with.

Calls only ``oracle/`` (and the seeded input builders of ``synth``): each
target is solved by the oracle's BiCGstab over its host FFT matvec in
complex128 (that matvec is pinned to the direct pair sum in
tests/test_oracle_fft_baseline.py) to a relative residual of 1e-10, and the
efficiencies of the solution (the oracle's cross-section sums) are written to
``oracle_full_size.txt`` beside this script, one line per right-hand side:

    name pol Q_ext Q_abs Q_sca rel_resid iterations

Run: ``python tests/golden/make_oracle_golden.py [name ...]`` (a few minutes
on 8 cores); with names, only those cases are recomputed and the other lines
of the file are kept.
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import dda, fft_baseline  # noqa: E402

# name -> (occupancy builder, m, size parameter x, orientation (beta, Theta, Phi))
CASES = {
    # the guide's worked example: Au block 32 x 64 x 64 (x along the incident
    # direction), N = 131072, m = 0.9656+1.8628i, x = 6.187304, Theta = Phi = beta = 0
    "block32x64x64": (lambda: np.ones((64, 64, 32), np.uint8), 0.9656 + 1.8628j, 6.187304, (0.0, 0.0, 0.0)),
    # the 64^3 sphere workload (N = 137,376), m = 1.5+0.1i, x = 10
    "sphere64": (lambda: synth.sphere_occupancy(64), 1.5 + 0.1j, 10.0, (0.4, 1.0, 0.3)),
}
# a mixed-box batch: ellipsoids in 32^3, 48^3 and 64^3 boxes, one random
# orientation each (seed CONFIG_SEED_BASE + 30); given as (occupancy, m, kd)
MIXED_BOXES = (32, 48, 64)
MIXED_SEED = synth.CONFIG_SEED_BASE + 30


def mixed_batch():
    """[(name, occ, m, kd, (beta, Theta, Phi))] of the mixed-box batch."""
    rng = np.random.default_rng(MIXED_SEED)
    tg = synth.mixed_box_targets(MIXED_BOXES, rng)
    ori = synth.uniform_orientations(len(tg), rng)
    return [(f"mixed{n}", occ, m, kd, tuple(o)) for n, (occ, m, kd), o in zip(MIXED_BOXES, tg, ori)]
OUT = os.path.join(HERE, "oracle_full_size.txt")


def case_inputs(name):
    """(occupancy, m, kd, (beta, Theta, Phi)) of a named case."""
    if name in CASES:
        build, m, x, ori = CASES[name]
        occ = build()
        return occ, m, x / dda.effective_radius(int(np.count_nonzero(occ))), ori
    for nm, occ, m, kd, ori in mixed_batch():
        if nm == name:
            return occ, m, kd, ori
    raise KeyError(name)


def all_names():
    return list(CASES) + [c[0] for c in mixed_batch()]


def solve_case(name, tol=1e-10):
    occ, m, kd, (beta, theta, phi) = case_inputs(name)
    r, comp, _ = dda.sites_from_occupancy(occ)
    khat, es, _ = dda.waves_for_orientation(beta, theta, phi)
    rows = []
    for pol, e in enumerate(es):
        ainv = dda.site_inverse_polarizability(comp, [m], kd, dda.ALPHA_LDR, khat, e)
        F = fft_baseline.FftDda(r, kd, ainv)
        E = dda.incident_field(r, kd, khat, e)
        P, info = F.solve(E, tol=tol)
        q = dda.cross_sections(kd, E, P, ainv)
        rows.append((name, pol, *q, info["rel_resid"], info["iters"]))
        print(rows[-1], flush=True)
    return rows


def read_golden(path=OUT):
    """{(name, pol): (Q_ext, Q_abs, Q_sca)} from the stored file."""
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            v = line.split()
            out[(v[0], int(v[1]))] = tuple(float(t) for t in v[2:5])
    return out


def main(names):
    keep = []
    if names and os.path.exists(OUT):
        keep = [l.split() for l in open(OUT) if l.strip() and not l.startswith("#") and l.split()[0] not in names]
        keep = [(v[0], int(v[1]), float(v[2]), float(v[3]), float(v[4]), float(v[5]), int(v[6])) for v in keep]
    rows = list(keep)
    for name in names or all_names():
        rows += solve_case(name)
    order = {n: i for i, n in enumerate(all_names())}
    rows.sort(key=lambda row: (order.get(row[0], 99), row[1]))
    with open(OUT, "w") as f:
        f.write("# written by make_oracle_golden.py (oracle BiCGstab over its complex128 FFT matvec, tol 1e-10)\n")
        f.write("# name pol Q_ext Q_abs Q_sca rel_resid iterations\n")
        for row in rows:
            f.write(f"{row[0]} {row[1]} {row[2]:.12e} {row[3]:.12e} {row[4]:.12e} {row[5]:.3e} {row[6]}\n")


if __name__ == "__main__":
    main(sys.argv[1:])
