#!/usr/bin/env python3
"""Benchmark of the DDA solve hot path on one MI355X.

Headline workload: sphere inscribed in a 128^3 box (N = 1,099,136 dipoles),
doubled FFT grid 256^3, m = 1.33 + 0.01i, size parameter x = 20 (k d =
0.3124), LDR polarizability, 16 random orientations x 2 orthogonal
polarizations = 32 right-hand sides sharing one Green's-tensor spectrum.  One
step is the whole hot path for that batch: the incident fields, the
FP32-matvec BiCGstab with FP64 residual refinement to ||E - A P|| / ||E|| <=
1e-5, the cross sections, and the scattering amplitudes at 37 angles in two
planes of every orientation.  The one-off target set-up and Green's-tensor FFT
are outside the timed region.  ``value`` = converged solves per second.

Also reported: the per-pass matvec roofline at 32 rhs (HIP events on the
context's stream, algorithmic bytes of each pass) and the matvec at 2, 8 and
32 rhs; the 64^3 sphere (2 rhs, with an all-FP64 comparison, moments and near
field); orientational averaging; the mixed-box batch; the learned initial
guess; and the CPU oracle timed on a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0  # dense BF16 MFMA
METRIC = "converged DDA solves/s at resid 1e-5 (learned vs plain); matvec % HBM peak"

# HBM bytes per launch from rocprofv3 counter runs of `bench.py
# --matvec-only --matvec-box 128|64`: reads = 32, 64 and 128 bytes times the
# L2's memory read requests of each size (TCC_EA0_RDREQ_32B/_64B/_128B),
# writes = 64 bytes times TCC_EA0_WRREQ_64B plus 32 bytes times the other
# write requests (median of 6 dispatches).  Valid only while the kernel's
# sources are the ones measured (SHA-256 prefix of their concatenation).
# Keyed by kernel name and rhs count of the launch; the summaries with the
# commands are profiles/matvec_traffic_box128_grid256.md and
# profiles/matvec_traffic_box64_grid128.md.
_CT_SOURCES = ("paper_1002_1505_amd/csrc/kernels_ct.hip", "paper_1002_1505_amd/csrc/dda_device.h")
MEASURED_TRAFFIC = {
    ("k_zpass5_ct<8, true>", 32): {"sources": _CT_SOURCES, "sha256": "446d6f046b54805c",
                                   "read_bytes": 8138509312, "write_bytes": 8247242112},
    ("k_zpass4_ct<float, 64, 16, true>", 2): {"sources": _CT_SOURCES, "sha256": "446d6f046b54805c",
                                               "read_bytes": 64458048, "write_bytes": 50331648},
}


def sources_digest(paths):
    """SHA-256 prefix (16 hex digits) of the concatenated files, paths relative to this file; None if one is missing."""
    import hashlib

    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        for p in paths:
            with open(os.path.join(root, p), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, nrhs: int):
    """HBM bytes per launch of `kernel` if its sources are unchanged since the counters were taken, else None."""
    m = MEASURED_TRAFFIC.get((kernel, nrhs))
    if m is None or sources_digest(m["sources"]) != m["sha256"]:
        return None
    return float(m["read_bytes"] + m["write_bytes"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--orientations", type=int, default=16, help="orientations of the headline sphere (2 rhs each)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target wall time of the CPU sample")
    ap.add_argument("--no-c2", action="store_true", help="skip the 64^3 sphere leg")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-guess comparison")
    ap.add_argument("--no-orient", action="store_true", help="skip the orientational-average leg")
    ap.add_argument("--no-c3", action="store_true", help="skip the mixed-box batch leg")
    ap.add_argument("--c3-orientations", type=int, default=64)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run three plain 256 MiB device copies (reference kernel for HBM byte counters)")
    ap.add_argument("--train-targets", type=int, default=33,
                    help="training targets; each sweep records (train-orient - 1) x 2 fields (33 x 31 x 2 = 2046)")
    ap.add_argument("--train-orient", type=int, default=32)
    ap.add_argument("--nn-width", type=int, default=16, choices=[16, 32, 64],
                    help="hidden channels (width 64, depth 10: the 940k-parameter network)")
    ap.add_argument("--nn-depth", type=int, default=4)
    ap.add_argument("--history", type=int, default=4, help="solutions kept per slot for the least-squares guess (at most 4)")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--eval-targets", type=int, default=2)
    ap.add_argument("--sweep", type=int, default=32)
    ap.add_argument("--solver", choices=["bicgstab", "bicgstab2"], default="bicgstab2",
                    help="Krylov solver of the headline and mixed-batch legs (bicgstab2: BiCGstab(2), the "
                         "guide's default PBCGS2)")
    ap.add_argument("--matvec-only", action="store_true",
                    help="only the headline target's FP32 matvec at 32 rhs (reps launches of each pass), for "
                         "profiler runs; prints the per-pass times and exits")
    ap.add_argument("--reps", type=int, default=5, help="launches per pass in --matvec-only")
    ap.add_argument("--matvec-box", type=int, choices=[64, 128], default=128,
                    help="--matvec-only target: the 128^3 sphere at 32 rhs or the 64^3 sphere at 2 rhs")
    return ap.parse_args()


SOLVERS = {"bicgstab": 0, "bicgstab2": 1}


def pass_names(P, ctx, n, prec_name="float"):
    """Kernel names of the three matvec passes for the context's current FP32 shape."""
    sh = ctx.get_shape(0, P.DDA_FP32)
    if sh["ct"] & 1:
        grp = "true" if sh["ct"] & 8 else "false"  # class-grouped slab
        zname = {0: f"k_zpass_ct<float, {n}, {sh['tx']}>", 1: f"k_zpass2_ct<float, {n}, {sh['tx']}, 8>",
                 2: f"k_zpass3_ct<float, {n}, {sh['tx']}>",
                 3: f"k_zpass4_ct<float, {n}, {sh['tx']}, {grp}>",
                 4: f"k_zpass5_ct<{sh['tx']}, {grp}>"}[sh["zrb"]]
        if n == 128 and grp == "true":
            iname = "k_pinvq_ct<0, 0|1|2|3>"  # four planes of one class per block
        else:
            iname = "k_pinv3_ct" if sh["ct"] & 4 else "k_pinv_ct"
            iname = f"{iname}<float, {n}, 0, 0|1|2|3, {grp}>"
        return [f"k_pfwd_ct<float, {n}, 0|2, {grp}>", zname, iname], sh
    return ["k_plane_fwd<float>", "k_zpass<float>", "k_plane_inv<float, 0>"], sh


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {a.gpus} is not supported "
              "(the right-hand sides would shard across GPUs with no communication inside a solve)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1002_1505_amd as P
    import synth

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if a.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = P.Context(0, stream=stream.cuda_stream)
    solver = SOLVERS[a.solver]

    # headline: the 128^3 sphere, 16 orientations x 2 polarizations
    n, x, m = 128, 20.0, 1.33 + 0.01j
    if a.matvec_only and a.matvec_box == 64:
        n, x, m = 64, 10.0, 1.5 + 0.1j
    occ = synth.sphere_occupancy(n)
    N = int(occ.sum())
    aeff = (3.0 * N / (4.0 * np.pi)) ** (1.0 / 3.0)
    kd = x / aeff
    t0 = time.time()
    ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
    ctx.build_green_fft(P.DDA_FP32 | P.DDA_FP64)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    if a.matvec_only:
        nr = 2 * a.orientations if n == 128 else 2
        ms, by = ctx.profile_matvec(0, nrhs=nr, prec=P.DDA_FP32, reps=a.reps)
        names, sh = pass_names(P, ctx, n)
        print(json.dumps({"matvec_only": True, "nrhs": nr, "reps": a.reps, "kernels": names, "shape": sh,
                          "pass_ms": [round(float(v), 5) for v in ms], "bytes": [float(v) for v in by],
                          "pass_GBs": [round(float(v), 1) for v in by / (ms * 1e-3) / 1e9]}), flush=True)
        ctx.close()
        return
    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 4)
    ori = synth.uniform_orientations(a.orientations, rng)
    kh, e0, n_tf, e_tf = [], [], [], []
    th = np.deg2rad(np.arange(0, 181, 5.0))
    thetas = np.concatenate([th, th])
    phis = np.concatenate([np.zeros_like(th), np.full_like(th, np.pi / 2)])
    for b, t, p in ori:
        k2, e2 = P.orientation_waves(b, t, p)
        kh += list(k2)
        e0 += list(e2)
        nt, et = P.scattering_frame(thetas, phis, P.lab_frame(b, t, p))
        n_tf.append(nt)
        e_tf.append(et)
    nrhs = len(kh)
    # each rhs's own orientation's 74 directions, in the target frame
    n_tf = np.stack([n_tf[i // 2] for i in range(nrhs)])
    e_tf = np.stack([e_tf[i // 2] for i in range(nrhs)])

    def step():
        _, st, status = ctx.solve(kh, e0, tol=1e-5, prec=P.DDA_SOLVE_FP32_REFINE, want_p=False, solver=solver)
        q = ctx.cross_sections(nrhs)
        f = ctx.amplitudes_per_rhs(nrhs, n_tf, e_tf)  # (rhs, its orientation's 74 directions, 2)
        return st, q, f

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(a.steps):
        st, q, f = step()
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = ctx.last_timing()
    nsolve = nrhs * a.steps
    conv = sum(1 for st in stats for s in st if s["status"] == 0 and s["rel_resid"] <= 1e-5)
    value = conv / dt
    # per-pass matvec roofline at the batch size of the headline solve, and
    # the whole matvec at 2, 8 and 32 rhs (FP32, the solve's launch shapes)
    names, sh = pass_names(P, ctx, n)
    mv = {}
    for nr in (2, 8, nrhs):
        ms, by = ctx.profile_matvec(0, nrhs=nr, prec=P.DDA_FP32, reps=5 if nr > 8 else 10)
        mv[nr] = (ms, by)
    ms, by = mv[nrhs]
    dom = int(np.argmax(ms))
    gbs = by / (ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(dt / a.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 matvec / f64 refine",
        "data": "synthetic: seeded pseudosphere and orientations, no external data",
        "config": {
            "workload": f"sphere in {n}^3 box (N={N}), FFT grid {2 * n}^3, m=1.33+0.01i, x={x}, LDR, "
                        f"{a.orientations} random orientations x 2 polarizations = {nrhs} rhs in one solve, "
                        f"{'BiCGstab(2)' if solver else 'BiCGstab'}, FP32 matvec + FP64 refinement, tol 1e-5, "
                        "cross sections and 74-direction amplitudes per orientation",
            "global_batch": nrhs,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": names[dom],
            "achieved": round(float(gbs[dom]), 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(float(gbs[dom]) / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(names[dom], nrhs),
            "bytes_per_launch": float(by[dom]),
            "avg_launch_ms": round(float(ms[dom]), 5),
            "nrhs": nrhs,
            "shape": sh,
        },
        "matvec": {
            str(nr): {"pass_ms": [round(float(v), 5) for v in mv[nr][0]],
                      "pass_GBs": [round(float(v), 1) for v in mv[nr][1] / (mv[nr][0] * 1e-3) / 1e9],
                      "total_ms": round(float(mv[nr][0].sum()), 5),
                      "GBs": round(float(mv[nr][1].sum() / (mv[nr][0].sum() * 1e-3) / 1e9), 1),
                      "frac_hbm": round(float(mv[nr][1].sum() / (mv[nr][0].sum() * 1e-3) / 1e9) / HBM_PEAK_GBS, 4)}
            for nr in mv},
        "solve": {
            "solver": a.solver,
            "matvecs_mean": round(float(np.mean([s["matvecs"] for s in stats[-1]])), 2),
            "iters_mean": round(float(np.mean([s["iters"] for s in stats[-1]])), 2),
            "iters_max": int(max(s["iters"] for s in stats[-1])),
            "outer": sorted(set(s["outer"] for s in stats[-1])),
            "rel_resid_max": max(s["rel_resid"] for s in stats[-1]),
            "converged": f"{conv}/{nsolve}",
            "ms_fp32_inner": round(tim["ms_mv32"], 3),
            "ms_fp64_residual": round(tim["ms_mv64"], 3),
            "Q_mean": [round(float(v), 6) for v in q.mean(axis=0)],
            "S11_forward_mean": round(float(np.mean(np.abs(f[:, 0, :]) ** 2)), 3),
        },
        "setup_s": round(setup_s, 3),
    }
    if not a.no_c2:
        out["c2"] = sphere64(P, ctx, synth, a)
    if not a.no_orient:
        occ64 = synth.sphere_occupancy(64)
        kd64 = 10.0 / ((3.0 * int(occ64.sum()) / (4.0 * np.pi)) ** (1.0 / 3.0))
        out["orient_avg"] = orientation_average(P, ctx, a, occ64, kd64, 1.5 + 0.1j)
    if not a.no_c3:
        out["c3"] = mixed_batch(P, ctx, synth, n_orient=a.c3_orientations, solver=solver)
    if not a.no_learned:
        out["learned"] = learned_vs_plain(P, ctx, a)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(occ, kd, m, stats[-1], a.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


def sphere64(P, ctx, synth, a, steps=10):
    """The 64^3 sphere (N = 137,376, grid 128^3, m = 1.5+0.1i, x = 10, LDR),
    one orientation x 2 polarizations: solves/s with FP32 matvecs and FP64
    refinement and all-FP64, the per-pass matvec roofline at 2 rhs, Q_pha,
    Q_bk and the eta = 0.5 moments, and E and B along a track."""
    import torch

    n, x, m = 64, 10.0, 1.5 + 0.1j
    occ = synth.sphere_occupancy(n)
    N = int(occ.sum())
    kd = x / ((3.0 * N / (4.0 * np.pi)) ** (1.0 / 3.0))
    ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
    ctx.build_green_fft(P.DDA_FP32 | P.DDA_FP64)
    khat, e0 = P.orientation_waves(0.0, 0.0, 0.0)
    L = P.lab_frame(0.0, 0.0, 0.0)
    th = np.deg2rad(np.arange(0, 181, 5.0))
    n_tf, e_tf = P.scattering_frame(np.concatenate([th, th]),
                                    np.concatenate([np.zeros_like(th), np.full_like(th, np.pi / 2)]), L)

    def step(prec):
        _, st, status = ctx.solve(khat, e0, tol=1e-5, prec=prec, want_p=False)
        return st, ctx.cross_sections(2), ctx.amplitudes(2, n_tf, e_tf)

    step(P.DDA_SOLVE_FP32_REFINE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st, q, f = step(P.DDA_SOLVE_FP32_REFINE)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step(P.DDA_SOLVE_FP64)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k64 = max(2, steps // 4)
    for _ in range(k64):
        st64, q64, f64 = step(P.DDA_SOLVE_FP64)
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t1
    q_rel = float(np.max(np.abs(q - q64) / np.abs(q64)))
    n_q, w_q = P.scattering_quadrature(x, 0.5, L)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    mom = ctx.scattering_moments(2, n_q, w_q)
    torch.cuda.synchronize()
    ms_mom = 1e3 * (time.perf_counter() - t2)
    track = np.linspace([-1.5 * n / 2, 0.25, 0.25], [1.5 * n / 2, 0.25, 0.25], 481)
    ctx.near_field(2, track)  # warm-up
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    Enf, Bnf = ctx.near_field(2, track)
    torch.cuda.synchronize()
    ms_nf = 1e3 * (time.perf_counter() - t2)
    e2 = np.sum(np.abs(Enf) ** 2, axis=-1).mean(axis=0)
    inside = np.abs(track[:, 0]) < 0.95 * n / 2
    ms, by = ctx.profile_matvec(0, nrhs=2, prec=P.DDA_FP32, reps=20)
    names, sh = pass_names(P, ctx, n)
    dom = int(np.argmax(ms))
    gbs = by / (ms * 1e-3) / 1e9
    ms64, by64 = ctx.profile_matvec(0, nrhs=2, prec=P.DDA_FP64, reps=5)
    # the same FP32 passes at 8 and 32 rhs (one solve of a sweep or a batch)
    by_nr = {2: (ms, by)}
    for nr in (8, 32):
        by_nr[nr] = ctx.profile_matvec(0, nrhs=nr, prec=P.DDA_FP32, reps=10)
    conv = sum(1 for s in st if s["status"] == 0 and s["rel_resid"] <= 1e-5)
    return {
        "workload": f"sphere in {n}^3 box (N={N}), FFT grid {2 * n}^3, m=1.5+0.1i, x={x}, LDR, 1 orientation x 2 "
                    "polarizations, FP32 matvec + FP64 refinement, tol 1e-5, cross sections and 74 amplitudes",
        "solves_per_s": round(2 * steps / dt, 3),
        "converged": f"{conv}/2",
        "iters": [s["iters"] for s in st],
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": round(float(gbs[dom]), 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(float(gbs[dom]) / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(names[dom], 2), "bytes_per_launch": float(by[dom]),
                     "avg_launch_ms": round(float(ms[dom]), 5), "shape": sh},
        "matvec": {"nrhs": 2, "pass_ms": [round(float(v), 5) for v in ms],
                   "pass_GBs": [round(float(v), 1) for v in gbs], "total_ms": round(float(ms.sum()), 5),
                   "GBs": round(float(by.sum() / (ms.sum() * 1e-3) / 1e9), 1),
                   "frac_hbm": round(float(by.sum() / (ms.sum() * 1e-3) / 1e9) / HBM_PEAK_GBS, 4),
                   "fp64_total_ms": round(float(ms64.sum()), 5),
                   "fp64_GBs": round(float(by64.sum() / (ms64.sum() * 1e-3) / 1e9), 1),
                   "by_nrhs": {str(nr): {"pass_ms": [round(float(v), 5) for v in m_],
                                         "total_ms": round(float(m_.sum()), 5),
                                         "GBs": round(float(b_.sum() / (m_.sum() * 1e-3) / 1e9), 1),
                                         "frac_hbm": round(float(b_.sum() / (m_.sum() * 1e-3) / 1e9) / HBM_PEAK_GBS, 4)}
                               for nr, (m_, b_) in by_nr.items()}},
        "fp64_solve": {"solves_per_s": round(2 * k64 / dt64, 3), "iters": [s["iters"] for s in st64],
                       "max_rel_diff_Q_fp32refine_vs_fp64": q_rel},
        "Q": [list(map(float, qq)) for qq in q],
        "moments": {"ndir": int(len(w_q)), "eta": 0.5, "ms": round(ms_mom, 3),
                    "per_pol": [{"Qpha": round(float(mm["Qpha"]), 6), "Qbk": round(float(mm["Qbk"]), 6),
                                 "Qsca_quad": round(float(mm["Qsca_quad"]), 6), "cos": round(float(mm["cos"]), 6),
                                 "cos2": round(float(mm["cos2"]), 6)} for mm in mom]},
        "near_field": {"points": int(len(track)),
                       "track": "x from -1.5 to +1.5 sphere radii at y = z = 0.25, lattice units from the centroid",
                       "ms": round(ms_nf, 3), "site_fields_per_s": round(2 * len(track) * N / (ms_nf * 1e-3), 1),
                       "mean_E2_inside": round(float(e2[inside].mean()), 5),
                       "mean_E2_outside": round(float(e2[~inside].mean()), 5)},
    }


def mixed_batch(P, ctx, synth, boxes=(32, 32, 32, 48, 48, 48, 64, 64), n_orient=64, max_iter=5000, solver=1):
    """Seeded random ellipsoids in 32^3, 48^3 and 64^3 boxes (axis ratios
    1 : U[1,2] : U[1,3], random rotation), Re m ~ U[1.2, 1.8], Im m ~
    log-U[0.001, 0.3], |m| k d ~ U[0.3, 0.8], LDR; n_orient uniform random
    orientations x 2 polarizations per target, all in one solve call (one
    graph over every target's group), launch shapes from the autotuner."""
    import tempfile

    import torch

    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 3)
    tgt = synth.mixed_box_targets(boxes, rng)
    for t, (occ, m, kd) in enumerate(tgt):
        if t == 0:
            ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
        else:
            ctx.add_target(occ, [m], kd, P.DDA_ALPHA_LDR)
    ctx.build_green_fft(P.DDA_FP32 | P.DDA_FP64)
    kh, e0, tg = [], [], []
    for t in range(len(tgt)):
        for b, th, ph in synth.uniform_orientations(n_orient, rng):
            k2, e2 = P.orientation_waves(b, th, ph)
            kh += list(k2)
            e0 += list(e2)
            tg += [t, t]
    nrhs = len(kh)
    t0 = time.perf_counter()
    with tempfile.TemporaryDirectory() as d:
        ctx.autotune(2 * n_orient, os.path.join(d, "tune.json"))
    tune_s = time.perf_counter() - t0
    # warm-up: workspaces and graphs, a few iterations
    ctx.solve(kh, e0, targets=tg, tol=1e-5, want_p=False, max_iter=8, solver=solver)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st, _ = ctx.solve(kh, e0, targets=tg, tol=1e-5, want_p=False, max_iter=max_iter, solver=solver)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sel = [[i for i in range(nrhs) if tg[i] == t] for t in range(len(tgt))]
    conv = sum(1 for s in st if s["status"] == 0 and s["rel_resid"] <= 1e-5)
    iters = [float(np.mean([st[i]["iters"] for i in sel[t]])) for t in range(len(tgt))]
    return {
        "workload": f"{len(tgt)} random ellipsoids in boxes {list(boxes)}, {n_orient} orientations x 2 "
                    f"polarizations each, LDR, {'BiCGstab(2)' if solver else 'BiCGstab'}, FP32 matvec + FP64 "
                    "refinement, tol 1e-5, one solve call, autotuned launch shapes",
        "solves": nrhs,
        "converged": f"{conv}/{nrhs}",
        "solves_per_s": round(nrhs / dt, 2),
        "solve_s": round(dt, 3),
        "autotune_s": round(tune_s, 2),
        "mean_iters_by_target": [round(v, 1) for v in iters],
        "mean_matvecs_by_target": [round(float(np.mean([st[i]["matvecs"] for i in sel[t]])), 1)
                                   for t in range(len(tgt))],
        "median_target_iters": round(float(np.median(iters)), 1),
        "m_kd": [[round(m.real, 3), round(m.imag, 4), round(kd, 4), round(abs(m) * kd, 3)] for _, m, kd in tgt],
        "sites": [int(o.sum()) for o, _, _ in tgt],
    }


def orientation_average(P, ctx, a, occ, kd, m, counts=(2, 5, 8), reps=3):
    """Orientationally averaged efficiencies of the bench sphere with the
    Clausius-Mossotti polarizability (the Phi combination needs a
    polarization-independent 1/alpha): NBETA x NTHETA (beta, Theta) pairs
    solved in one batch of 2 NBETA NTHETA right-hand sides, NPHI rotations
    each from dda_cross_sections_phi, weights from dda_orientation_samples."""
    import torch

    ctx.set_target(occ, [m], kd, P.DDA_ALPHA_CM)
    ctx.build_green_fft(P.DDA_FP32 | P.DDA_FP64)
    lims = np.deg2rad([0, 360, 0, 180, 0, 360])
    b, t, p, w = P.orientation_samples(lims, counts)
    kh, e0, coeffs = [], [], []
    for be in b:
        for th in t:
            k2, e2 = P.orientation_waves(be, th, p[0])
            kh += list(k2)
            e0 += list(e2)
            coeffs.append(P.phi_coefficients(be, th, p[0], p))
    coeffs = np.stack(coeffs)
    nrhs = len(kh)
    ctx.solve(kh, e0, tol=1e-5, want_p=False)  # warm-up (workspaces, graph)
    torch.cuda.synchronize()
    t_solve = t_phi = 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        _, st, _ = ctx.solve(kh, e0, tol=1e-5, want_p=False)
        t1 = time.perf_counter()
        q = ctx.cross_sections_phi(coeffs)
        t2 = time.perf_counter()
        t_solve += t1 - t0
        t_phi += t2 - t1
    q = q.reshape(len(b), len(t), len(p), 2, 3)
    qavg = np.tensordot(w, q, axes=([0, 1, 2], [0, 1, 2]))
    norient = len(b) * len(t) * len(p)
    conv = sum(1 for s in st if s["status"] == 0 and s["rel_resid"] <= 1e-5)
    return {
        "workload": f"{counts[0]} beta x {counts[1]} Theta (Simpson in cos Theta) x {counts[2]} Phi over the full "
                    f"ranges, bench sphere with CM polarizability, {nrhs} rhs in one batch, tol 1e-5",
        "orientations": norient,
        "solves": nrhs,
        "converged": f"{conv}/{nrhs}",
        "orientations_per_s": round(norient * reps / (t_solve + t_phi), 2),
        "solves_per_s": round(nrhs * reps / t_solve, 2),
        "ms_solve_batch": round(1e3 * t_solve / reps, 3),
        "ms_phi_combination": round(1e3 * t_phi / reps, 3),
        "mean_iters": round(float(np.mean([s["iters"] for s in st])), 2),
        "Q_avg": [[round(float(v), 6) for v in qq] for qq in qavg],
    }


def _aggregate_problem(synth, rng):
    occ = synth.aggregate_occupancy(64, rng)
    N = int(occ.sum())
    aeff = (3.0 * N / (4.0 * np.pi)) ** (1.0 / 3.0)
    x = rng.uniform(2.0, 10.0)
    m = complex(rng.uniform(1.3, 1.7), rng.uniform(0.01, 0.1))
    return occ, m, x / aeff


def learned_vs_plain(P, ctx, a):
    """Learned initial guess on porous aggregates in a 64^3 box (seeded
    Gaussian-random-field targets, fill 0.3, m = U[1.3,1.7] + i U[0.01,0.1],
    x = U[2,10]).  Training fields come from orientation sweeps (uniform in
    cos Theta, random beta, Phi) of held-in targets: each solve after the
    first starts from the least-squares guess over the last `history`
    solutions and is recorded.  Evaluation runs sweeps of held-out targets
    one orientation (2 polarizations) per solve, with P0 = 0, the previous
    orientation's P, that P phase-shifted to the new direction, the
    least-squares guess, and the network's correction of it; every mode
    starts its sweep from P0 = 0 and is timed whole, guess cost included."""
    import torch

    import synth

    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 5)
    net = P.Net(ctx, width=a.nn_width, depth=a.nn_depth, seed=5)
    t0 = time.perf_counter()
    for _ in range(a.train_targets):
        occ, m, kd = _aggregate_problem(synth, rng)
        ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
        ori = synth.theta_sweep(a.train_orient, beta=rng.uniform(0, 2 * np.pi), phi=rng.uniform(0, 2 * np.pi))
        for i, (b, t, p) in enumerate(ori):
            kh, ee = P.orientation_waves(b, t, p)
            ctx.solve(kh, ee, tol=1e-5, want_p=False, history=a.history,
                      guess=P.DDA_GUESS_ZERO if i == 0 else P.DDA_GUESS_PROJECT)
            if i:
                net.record()
    gen_s = time.perf_counter() - t0
    print(f"[learned] {net.num_samples} training fields in {gen_s:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    loss0 = loss = None
    for ep in range(a.epochs):
        loss = net.train(epochs=1, batch=4, lr=1e-3)
        loss0 = loss if loss0 is None else loss0
        print(f"[learned] epoch {ep + 1}/{a.epochs} loss {loss:.4f} ({time.perf_counter() - t0:.1f} s)",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    net.attach()
    modes = (("zero", P.DDA_GUESS_ZERO), ("prev", P.DDA_GUESS_PREV), ("prev_shift", P.DDA_GUESS_PREV_SHIFT),
             ("project", P.DDA_GUESS_PROJECT), ("nn", P.DDA_GUESS_NN))
    res = {m: [0, 0.0, 0] for m, _ in modes}  # iters, seconds, converged solves
    resid = {m: [] for m, _ in modes}
    guess_ms = {m: 0.0 for m, _ in modes}
    for _ in range(a.eval_targets):
        occ, m, kd = _aggregate_problem(synth, rng)
        ori = synth.theta_sweep(a.sweep, beta=rng.uniform(0, 2 * np.pi), phi=rng.uniform(0, 2 * np.pi))
        waves = [P.orientation_waves(b, t, p) for b, t, p in ori]
        for mode, g in modes:
            # every mode starts from the same state: the target defined anew
            # (which clears the slots' history of earlier solutions), its
            # spectrum built and one warm-up solve, outside the timed sweep
            ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
            ctx.build_green_fft(P.DDA_FP32 | P.DDA_FP64)
            ctx.solve(waves[0][0], waves[0][1], want_p=False)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for i, (kh, ee) in enumerate(waves):
                gg = P.DDA_GUESS_ZERO if i == 0 else g
                _, st, _ = ctx.solve(kh, ee, tol=1e-5, guess=gg, want_p=False, history=a.history)
                res[mode][0] += sum(s["iters"] for s in st)
                res[mode][2] += sum(1 for s in st if s["status"] == 0 and s["rel_resid"] <= 1e-5)
                if i:
                    resid[mode] += [s["guess_resid"] for s in st]
                    guess_ms[mode] += ctx.last_timing().get("ms_guess", 0.0)
            torch.cuda.synchronize()
            res[mode][1] += time.perf_counter() - t1
            print(f"[learned] {mode}: {time.perf_counter() - t1:.2f} s", file=sys.stderr, flush=True)
    n_solves = 2 * a.sweep * a.eval_targets
    out = {
        "workload": f"porous aggregates in 64^3 box, {a.train_targets} training targets x {a.train_orient}-orientation "
                    f"sweeps x 2 pol ({net.num_samples} recorded fields), {a.eval_targets} held-out targets x "
                    f"{a.sweep}-orientation sweeps x 2 pol, one orientation per solve, tol 1e-5",
        "net": f"width {a.nn_width}, depth {a.nn_depth}, {net.num_params} params, BF16 MFMA",
        "history": a.history,
        "train_loss_first_epoch": round(loss0, 4),
        "train_loss": round(loss, 4),
        "gen_s": round(gen_s, 2),
        "train_s": round(train_s, 2),
        "epochs": a.epochs,
    }
    for mode in res:
        it, sec, conv = res[mode]
        out[mode] = {"solves_per_s": round(conv / sec, 3), "mean_iters": round(it / n_solves, 2),
                     "converged": f"{conv}/{n_solves}",
                     "mean_guess_resid": round(float(np.mean(resid[mode])), 4) if resid[mode] else 1.0,
                     "guess_ms_per_solve": round(guess_ms[mode] / max(1, n_solves // 2 - a.eval_targets), 3)}
    # the network's kernels against the BF16 MFMA roof (device-resident
    # pseudo-random inputs on the same box, 2 samples = the 2 polarizations)
    f_ms, b_ms, gflop = net.profile(64, 2, 10)
    out["net_roofline"] = {"bound": "mfma", "achieved": round(gflop / f_ms, 1), "peak": BF16_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(gflop / f_ms / BF16_PEAK_TFLOPS, 4),
                           "forward_ms_2_samples": round(f_ms, 4), "backward_ms_2_samples": round(b_ms, 4),
                           "forward_gflop": round(gflop, 2)}
    for base in ("zero", "prev", "prev_shift", "project"):
        out[f"nn_vs_{base}"] = round(out["nn"]["solves_per_s"] / out[base]["solves_per_s"], 3)
    net.close()
    return out


def host_info():
    """Host cores the CPU baselines ran on: logical CPUs, the process's CPU
    affinity, and the processor model (from /proc/cpuinfo, else lscpu)."""
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    if not model:
        try:
            txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
            model = next((l.split(":", 1)[1].strip() for l in txt.splitlines() if l.startswith("Model name")), "")
        except (OSError, subprocess.SubprocessError):
            pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model or platform.processor()}


def cpu_baseline(occ, kd, m, stats, seconds):
    """The oracle's direct O(N^2) FP64 matvec on a bounded sample of rows of
    the headline workload, extrapolated to full solves: a solve costs as many
    matvecs as the GPU solve took (its FP32 and FP64 products counted as FP64
    oracle products)."""
    from oracle import dda

    r, comp, _ = dda.sites_from_occupancy(occ)
    n = len(r)
    khat, e = np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
    ainv = dda.site_inverse_polarizability(comp, [m], kd, dda.ALPHA_LDR, khat, e)
    rng = np.random.default_rng(0)
    x = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    rows = rng.choice(n, size=64, replace=False)
    t0 = time.perf_counter()
    dda.matvec_rows(r, kd, ainv, x, rows)
    t_probe = time.perf_counter() - t0
    nrows = int(min(n, max(64, 64 * seconds / max(t_probe, 1e-6))))
    rows = rng.choice(n, size=nrows, replace=False)
    t0 = time.perf_counter()
    dda.matvec_rows(r, kd, ainv, x, rows)
    t_rows = time.perf_counter() - t0
    t_matvec = t_rows * n / nrows
    mv_per_solve = float(np.mean([s["matvecs"] for s in stats]))
    t_solve = t_matvec * mv_per_solve
    return {
        "value": round(1.0 / t_solve, 10),
        "unit": "solves/s",
        "cores": dda.threads(),
        "kind": "oracle",
        "sample": f"direct O(N^2) FP64 matvec on {nrows} of {n} rows ({t_rows:.1f} s wall), extrapolated to "
                  f"{n} rows x {mv_per_solve:.0f} matvecs per solve",
        "host": host_info(),
        "matvec_s_extrapolated": round(t_matvec, 1),
        "fft_host": fft_host_baseline(r, kd, ainv, x, mv_per_solve, dda.threads()),
        "other_sizes": oracle_sizes(t_rows / (nrows * n)),
    }


def oracle_sizes(s_per_pair):
    """The oracle at the other sizes: the dense LU solve of the 16-diameter
    sphere (N = 2,176) timed in full, and the direct matvec of the 64^3
    sphere extrapolated from the per-pair cost measured above."""
    import synth
    from oracle import dda

    occ = synth.sphere_occupancy(16)
    r, comp, _ = dda.sites_from_occupancy(occ)
    kd = 4.0 / dda.effective_radius(len(r))
    ainv = dda.site_inverse_polarizability(comp, [1.5 + 0.1j], kd, dda.ALPHA_LDR, np.array([1.0, 0, 0]),
                                           np.array([0, 1.0, 0]))
    E = dda.incident_field(r, kd, np.array([1.0, 0, 0]), np.array([0, 1.0, 0]))
    t0 = time.perf_counter()
    dda.solve_dense(r, kd, ainv, E)
    t_lu = time.perf_counter() - t0
    n2 = int(synth.sphere_occupancy(64).sum())
    return {
        "dense_lu_sphere16": {"sites": len(r), "s_per_solve": round(t_lu, 3)},
        "direct_sphere64_extrapolated": {"sites": n2, "matvec_s": round(s_per_pair * n2 * n2, 2)},
    }


def fft_host_baseline(r, kd, ainv, x, mv_per_solve, workers):
    """The FFT method on the host cores (numpy/scipy FFTs on the doubled grid,
    not the oracle): one full-size matvec in complex64 and in complex128 after
    a complex64 warm-up, extrapolated to the GPU solve's matvec count."""
    from oracle import fft_baseline

    out = {"kind": "host FFT-DDA (numpy/scipy FFT, BiCGstab matvec count of the GPU solve), not the oracle",
           "workers": workers}
    for i, (name, dt) in enumerate((("c64", np.complex64), ("c128", np.complex128))):
        t0 = time.perf_counter()
        F = fft_baseline.FftDda(r, kd, ainv, dtype=dt, workers=workers)
        setup = time.perf_counter() - t0
        if i == 0:
            F.matvec(x)
        t0 = time.perf_counter()
        F.matvec(x)
        tm = time.perf_counter() - t0
        out["grid"] = list(F.M)
        out[name] = {"setup_s": round(setup, 2), "matvec_s": round(tm, 4),
                     "solves_per_s": round(1.0 / (tm * mv_per_solve), 6)}
        del F
    out["sample"] = f"one full-size matvec per precision, extrapolated to {mv_per_solve:.0f} matvecs per solve"
    return out


if __name__ == "__main__":
    main()
