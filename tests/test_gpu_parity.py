"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Inputs are seeded and synthetic (``synth``); every expected value comes from
``oracle/``.  Bars: FP64 matvec 1e-12 relative, FP32 matvec 5e-6 relative
(FFT rounding of complex64 on grids up to 256^3), solves to the requested
residual 1e-5 checked with the oracle's own matvec, efficiencies within
1e-4 relative of the oracle's solution.
"""
import numpy as np
import pytest

import synth
from oracle import dda, scatter

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1002_1505_amd as P

    c = P.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _setup(ctx, occ, m_list, kd, kind, origin=None):
    import paper_1002_1505_amd as P

    kinds = {dda.ALPHA_CM: P.DDA_ALPHA_CM, dda.ALPHA_CM_RR: P.DDA_ALPHA_CM_RR, dda.ALPHA_LDR: P.DDA_ALPHA_LDR}
    ctx.set_target(occ, m_list, kd, kinds[kind], origin=origin)
    r, comp, idx = dda.sites_from_occupancy(occ, origin)
    return r, comp


CASES = [
    # name, occupancy builder, m list, kd
    ("cube8_two_materials", lambda: np.concatenate([np.ones((2, 2, 1), np.uint8), 2 * np.ones((2, 2, 1), np.uint8)], axis=2),
     [1.5 + 0.01j, 2.0 + 1.0j], 0.4),
    ("sphere_d8", lambda: synth.sphere_occupancy(8), [1.33 + 0.01j], 0.3),
    ("ellipsoid_12x16x10", lambda: synth.ellipsoid_occupancy((12, 16, 10), (11.0, 15.0, 9.5)), [1.7 + 0.1j], 0.5),
    ("ragged_aggregate_20x24x15", lambda: (np.random.default_rng(7).random((15, 24, 20)) < 0.4).astype(np.uint8),
     [1.4 + 0.05j], 0.35),
]


@pytest.mark.parametrize("name,build,m_list,kd", CASES, ids=[c[0] for c in CASES])
def test_matvec_small_vs_oracle(ctx, name, build, m_list, kd):
    import paper_1002_1505_amd as P

    occ = build()
    r, comp = _setup(ctx, occ, m_list, kd, dda.ALPHA_LDR)
    rng = np.random.default_rng(11)
    nr = 2
    x = rng.standard_normal((nr, len(r), 3)) + 1j * rng.standard_normal((nr, len(r), 3))
    ainv = np.array([[dda.inverse_polarizability(mm, kd, dda.ALPHA_CM) + 0.1 * s for mm in m_list] for s in range(nr)])
    y64 = ctx.matvec(x, ainv=ainv, prec=P.DDA_FP64)
    y32 = ctx.matvec(x, ainv=ainv, prec=P.DDA_FP32)
    # the eight lattice parity classes (x, y, z mod 2), which the FFT path
    # handles in separate blocks, and the box faces
    ri = np.rint(r - r.min(axis=0)).astype(int)
    cls = (ri[:, 0] & 1) + 2 * (ri[:, 1] & 1) + 4 * (ri[:, 2] & 1)
    edge = np.any((ri == 0) | (ri == ri.max(axis=0)), axis=1)
    for s in range(nr):
        ref = dda.matvec_direct(r, kd, ainv[s][comp - 1], x[s])
        scale = np.sqrt(np.mean(np.abs(ref) ** 2))
        for y, tol in ((y64[s], 1e-12), (y32[s], 5e-6)):
            assert _rel(y, ref) < tol, name
            # element-wise, per parity class and on the box faces
            assert np.abs(y - ref).max() / scale < 10 * tol, name
            for q in range(8):
                sel = cls == q
                if sel.any():
                    assert _rel(y[sel], ref[sel]) < 3 * tol, (name, q)
            assert _rel(y[edge], ref[edge]) < 3 * tol, name


def test_matvec_bilinear_symmetry(ctx):
    """x^T (A y) = y^T (A x): the FFT operator keeps A symmetric."""
    import paper_1002_1505_amd as P

    occ = synth.ellipsoid_occupancy((16, 12, 20), (15.0, 11.0, 19.0))
    r, comp = _setup(ctx, occ, [1.5 + 0.2j], 0.4, dda.ALPHA_LDR)
    rng = np.random.default_rng(3)
    xy = rng.standard_normal((2, len(r), 3)) + 1j * rng.standard_normal((2, len(r), 3))
    for prec, tol in ((P.DDA_FP64, 1e-13), (P.DDA_FP32, 2e-6)):
        A = ctx.matvec(xy, prec=prec)
        lhs = np.sum(xy[0] * A[1])
        rhs = np.sum(xy[1] * A[0])
        assert abs(lhs - rhs) / abs(lhs) < tol


def test_single_dipole_closed_form(ctx):
    """N = 1 in a 2x2x2 box: P = alpha E, Q_ext = 4 pi k Im(alpha) / (pi a_eff^2)."""
    import paper_1002_1505_amd as P

    occ = np.zeros((2, 2, 2), np.uint8)
    occ[0, 0, 0] = 1
    kd, m = 0.3, 1.5 + 0.2j
    ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
    khat, e = [1.0, 0, 0], [0, 1.0, 0]
    Pg, st, _ = ctx.solve([khat], [e], tol=1e-10, prec=P.DDA_SOLVE_FP64)
    alpha = 1 / dda.inverse_polarizability(m, kd, dda.ALPHA_LDR, khat, e)
    assert np.allclose(Pg[0][0], alpha * np.array(e), rtol=1e-10)
    q = ctx.cross_sections(1)
    aeff = dda.effective_radius(1)
    assert np.isclose(q[0, 0], 4 * np.pi * kd * alpha.imag / (np.pi * aeff ** 2), rtol=1e-10)


def _c1_problem():
    occ = synth.sphere_occupancy(16)
    r, comp, _ = dda.sites_from_occupancy(occ)
    x = 1.0
    kd = x / dda.effective_radius(len(r))
    return occ, r, comp, kd, x


@pytest.mark.parametrize("prec_name", ["fp64", "fp32_refine"])
def test_config1_sphere16_vs_oracle(ctx, prec_name):
    """Sphere D = 16 (N = 2176), m = 1.33+0.01i, x = 1, LDR, two polarizations:
    P to residual 1e-5, Q's within 1e-4, amplitudes at 37 angles x 2 planes."""
    import paper_1002_1505_amd as P

    occ, r, comp, kd, x = _c1_problem()
    assert len(r) == 2176
    m = 1.33 + 0.01j
    ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
    khat, es, L = dda.waves_for_orientation(0.0, 0.0, 0.0)
    prec = P.DDA_SOLVE_FP64 if prec_name == "fp64" else P.DDA_SOLVE_FP32_REFINE
    Pg, stats, status = ctx.solve([khat, khat], es, tol=1e-5, prec=prec)
    assert status == 0
    qg = ctx.cross_sections(2)
    th = np.deg2rad(np.arange(0, 181, 5.0))
    Ps_or = []
    for l, e in enumerate(es):
        ainv = dda.site_inverse_polarizability(comp, [m], kd, dda.ALPHA_LDR, khat, e)
        E = dda.incident_field(r, kd, khat, e)
        Po, info = dda.solve_iterative(r, kd, ainv, E, tol=1e-11)
        Ps_or.append(Po)
        rel, _ = dda.residual_norms(r, kd, ainv, E, Pg[l])
        assert rel <= 1e-5 and stats[l]["rel_resid"] <= 1e-5
        assert abs(rel - stats[l]["rel_resid"]) < 1e-7
        qo = np.array(dda.cross_sections(kd, E, Po, ainv))
        assert np.all(np.abs(qg[l] - qo) / np.abs(qo) < 1e-4), (qg[l], qo)
    # amplitudes: directions in the two scattering planes
    for phi in (0.0, np.pi / 2):
        ph = np.full_like(th, phi)
        n_lab, t_lab, p_lab = scatter.lab_direction_basis(th, ph)
        n_tf, t_tf, p_tf = n_lab @ L, t_lab @ L, p_lab @ L
        f = ctx.amplitudes(2, n_tf, np.concatenate([t_tf, p_tf], axis=1))  # (rhs, dir, m)
        fo = scatter.scattering_amplitudes(r, kd, Ps_or, th, ph, L)       # (dir, m, l)
        fg = np.transpose(f, (1, 2, 0))
        assert np.max(np.abs(fg - fo)) / np.max(np.abs(fo)) < 1e-4


def test_solve_fp32_refine_matches_fp64(ctx):
    """Mixed precision meets the FP64 residual bar and agrees with the all-FP64 solve."""
    import paper_1002_1505_amd as P

    occ = synth.sphere_occupancy(24)
    ctx.set_target(occ, [1.5 + 0.1j], 0.5, P.DDA_ALPHA_LDR)
    khat, es, L = dda.waves_for_orientation(0.3, 0.7, 1.1)
    P64, s64, _ = ctx.solve([khat, khat], es, prec=P.DDA_SOLVE_FP64)
    q64 = ctx.cross_sections(2)
    P32, s32, _ = ctx.solve([khat, khat], es, prec=P.DDA_SOLVE_FP32_REFINE)
    q32 = ctx.cross_sections(2)
    for l in range(2):
        assert s32[l]["rel_resid"] <= 1e-5 and s64[l]["rel_resid"] <= 1e-5
        assert _rel(P32[l], P64[l]) < 1e-4
    assert np.all(np.abs(q32 - q64) / np.abs(q64) < 1e-4)


def test_guesses_user_prev_and_fallback(ctx):
    import paper_1002_1505_amd as P

    occ = synth.sphere_occupancy(12)
    ctx.set_target(occ, [1.4 + 0.05j], 0.4, P.DDA_ALPHA_LDR)
    khat, es, L = dda.waves_for_orientation(0.0, 0.5, 0.0)
    P0, s0, _ = ctx.solve([khat, khat], es, prec=P.DDA_SOLVE_FP64, tol=1e-8)
    # exact guess: converged before any iteration
    P1, s1, _ = ctx.solve([khat, khat], es, prec=P.DDA_SOLVE_FP64, tol=1e-5, guess=P.DDA_GUESS_USER, p0=P0)
    assert all(s["iters"] == 0 for s in s1)
    # previous solution as guess
    P2, s2, _ = ctx.solve([khat, khat], es, prec=P.DDA_SOLVE_FP64, tol=1e-5, guess=P.DDA_GUESS_PREV)
    assert all(s["iters"] == 0 for s in s2)
    # a guess worse than zero is replaced by zero
    bad = [100 * p for p in P0]
    P3, s3, _ = ctx.solve([khat, khat], es, prec=P.DDA_SOLVE_FP64, tol=1e-5, guess=P.DDA_GUESS_USER, p0=bad)
    assert all(s["guess_resid"] == 1.0 and s["rel_resid"] <= 1e-5 for s in s3)


def test_batched_uneven_targets_match_single_solves(ctx):
    """Three targets of different boxes in one call give the same P as
    separate calls (per-rhs convergence masks, graph replay)."""
    import paper_1002_1505_amd as P

    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 3)
    occs = [synth.random_ellipsoid(n, rng)[0] for n in (16, 24, 32)]
    ms = [1.3 + 0.01j, 1.6 + 0.2j, 1.45 + 0.05j]
    kds = [0.4, 0.35, 0.3]
    ori = synth.uniform_orientations(2, rng)
    waves_k, waves_e, tg = [], [], []
    ctx.set_target(occs[0], [ms[0]], kds[0])
    for t in (1, 2):
        ctx.add_target(occs[t], [ms[t]], kds[t])
    for t in range(3):
        for b, th, ph in ori:
            kh, es, L = dda.waves_for_orientation(b, th, ph)
            for e in es:
                waves_k.append(kh)
                waves_e.append(e)
                tg.append(t)
    Pb, sb, _ = ctx.solve(waves_k, waves_e, targets=tg, prec=P.DDA_SOLVE_FP32_REFINE)
    qb = ctx.cross_sections(len(tg))
    for t in range(3):
        sel = [i for i in range(len(tg)) if tg[i] == t]
        ctx.set_target(occs[t], [ms[t]], kds[t])
        Ps, ss, _ = ctx.solve([waves_k[i] for i in sel], [waves_e[i] for i in sel], prec=P.DDA_SOLVE_FP32_REFINE)
        qs = ctx.cross_sections(len(sel))
        for k, i in enumerate(sel):
            assert sb[i]["rel_resid"] <= 1e-5
            assert _rel(Pb[i], Ps[k]) < 3e-5
            assert np.all(np.abs(qb[i] - qs[k]) / np.abs(qs[k]) < 1e-4)


def test_chunked_batch_matches_small_batches(ctx):
    """A batch whose slab outgrows the matvec chunk runs the three passes
    chunk by chunk on offset pointers: 24 rhs of a 48^3 sphere (FP32 slab
    10.6 MB per rhs, chunks of 19; FP64 21.2 MB, chunks of 9).  The matvec
    gives the same bits as three 8-rhs calls (which run whole), in FP32 and
    FP64; 24-rhs solves (the fused inner products and updates of the chunked
    passes, BiCGstab and BiCGstab(2)) match three 8-rhs solves."""
    import paper_1002_1505_amd as P

    occ = synth.sphere_occupancy(48)
    m, kd = 1.4 + 0.05j, 0.3
    ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
    r, comp, _ = dda.sites_from_occupancy(occ)
    rng = np.random.default_rng(synth.CONFIG_SEED_BASE + 29)
    x = rng.standard_normal((24, len(r), 3)) + 1j * rng.standard_normal((24, len(r), 3))
    ainv = [[dda.inverse_polarizability(m, kd, dda.ALPHA_CM)]] * 24
    for prec in (P.DDA_FP32, P.DDA_FP64):
        y = ctx.matvec(x, ainv=ainv, prec=prec)
        y8 = np.concatenate([ctx.matvec(x[i:i + 8], ainv=ainv[i:i + 8], prec=prec) for i in (0, 8, 16)])
        assert np.array_equal(y, y8), prec
    kh, ee = [], []
    for b, th, ph in synth.uniform_orientations(12, rng):
        k2, e2, _ = dda.waves_for_orientation(b, th, ph)
        kh += [k2, k2]
        ee += list(e2)
    for solver in (P.DDA_SOLVER_BICGSTAB, P.DDA_SOLVER_BICGSTAB2):
        Pb, sb, stb = ctx.solve(kh, ee, prec=P.DDA_SOLVE_FP32_REFINE, solver=solver)
        assert stb == 0
        qb = ctx.cross_sections(24)
        for i0 in (0, 8, 16):
            Ps, ss, sts = ctx.solve(kh[i0:i0 + 8], ee[i0:i0 + 8], prec=P.DDA_SOLVE_FP32_REFINE, solver=solver)
            assert sts == 0
            qs = ctx.cross_sections(8)
            for k in range(8):
                i = i0 + k
                assert sb[i]["rel_resid"] <= 1e-5
                assert _rel(Pb[i], Ps[k]) < 1e-6, (solver, i, sb[i], ss[k])
                assert np.all(np.abs(qb[i] - qs[k]) <= 1e-6 * np.abs(qs[k]))


def test_graph_and_eager_agree(ctx):
    import paper_1002_1505_amd as P

    occ = synth.sphere_occupancy(16)
    ctx.set_target(occ, [1.5 + 0.1j], 0.4)
    khat, es, L = dda.waves_for_orientation(0.2, 0.4, 0.6)
    Pg, sg, _ = ctx.solve([khat, khat], es, prec=P.DDA_SOLVE_FP32_REFINE)
    Pe, se, _ = ctx.solve([khat, khat], es, prec=P.DDA_SOLVE_FP32_REFINE, flags=P.DDA_NO_GRAPH)
    for l in range(2):
        assert sg[l]["iters"] == se[l]["iters"]
        assert _rel(Pg[l], Pe[l]) < 1e-6


def test_replay_depth_does_not_change_the_iterates(ctx):
    """The number of iterations per graph replay (and the replay queued
    ahead of each convergence poll) only changes when convergence is
    checked: iteration counts and solutions are the same for every depth."""
    import paper_1002_1505_amd as P

    occ = synth.sphere_occupancy(16)
    ctx.set_target(occ, [1.5 + 0.1j], 0.4)
    khat, es, L = dda.waves_for_orientation(0.7, 1.1, 0.2)
    ref, sref, _ = ctx.solve([khat, khat], es, prec=P.DDA_SOLVE_FP32_REFINE, graph_iters=4)
    for gi in (2, 6, 10):
        Pg, sg, _ = ctx.solve([khat, khat], es, prec=P.DDA_SOLVE_FP32_REFINE, graph_iters=gi)
        for l in range(2):
            assert sg[l]["iters"] == sref[l]["iters"], (gi, l)
            assert _rel(Pg[l], ref[l]) < 1e-12, (gi, l)


def test_shifted_previous_guess_vs_oracle(ctx):
    """Two consecutive orientations of a sweep (Theta step, both
    polarizations): the residual of the PREV and PREV_SHIFT guesses on the
    GPU equals the oracle's residual of the same guesses built from the
    oracle's own previous solution."""
    import paper_1002_1505_amd as P

    occ = synth.ellipsoid_occupancy((12, 16, 10), (11.0, 15.0, 9.5))
    m, kd = [1.5 + 0.05j], 0.5
    r, comp = _setup(ctx, occ, m, kd, dda.ALPHA_LDR)
    kp, ep, _ = dda.waves_for_orientation(0.4, 0.9, 0.3)
    kn, en, _ = dda.waves_for_orientation(0.4, 1.05, 0.3)

    def oracle_solve(kh, e):
        ainv = dda.site_inverse_polarizability(comp, m, kd, dda.ALPHA_LDR, kh, e)
        E = dda.incident_field(r, kd, kh, e)
        return ainv, E, dda.solve_dense(r, kd, ainv, E)

    expect = {"prev": [], "shift": []}
    for l in range(2):
        ap, _, Pp = oracle_solve(kp, ep[l])
        an = dda.site_inverse_polarizability(comp, m, kd, dda.ALPHA_LDR, kn, en[l])
        En = dda.incident_field(r, kd, kn, en[l])
        _, P0 = dda.shifted_previous_guess(r, kd, Pp, ap, an, kp, kn)
        y0 = dda.matvec_direct(r, kd, an, Pp)
        y1 = dda.matvec_direct(r, kd, an, P0)
        expect["prev"].append(np.linalg.norm(En - y0) / np.linalg.norm(En))
        expect["shift"].append(np.linalg.norm(En - y1) / np.linalg.norm(En))
    for name, guess in (("prev", P.DDA_GUESS_PREV), ("shift", P.DDA_GUESS_PREV_SHIFT)):
        ctx.solve([kp, kp], ep, prec=P.DDA_SOLVE_FP64, tol=1e-11, want_p=False)
        _, st, _ = ctx.solve([kn, kn], en, prec=P.DDA_SOLVE_FP64, tol=1e-5, guess=guess)
        for l in range(2):
            assert abs(st[l]["guess_resid"] - expect[name][l]) <= 1e-7 + 1e-6 * expect[name][l], (name, l)
            assert st[l]["rel_resid"] <= 1e-5
    # on this sweep step the phase shift improves on the unshifted previous solution
    assert sum(expect["shift"]) < sum(expect["prev"])


def test_projected_history_guess_vs_oracle(ctx):
    """Least-squares guess over the last three solutions of a sweep (history
    3): the GPU guess residual (FP32 basis and products, FP64 residual) equals
    the oracle's residual of its own projection."""
    import paper_1002_1505_amd as P

    occ = synth.ellipsoid_occupancy((12, 16, 10), (11.0, 15.0, 9.5))
    m, kd = [1.5 + 0.05j], 0.5
    r, comp = _setup(ctx, occ, m, kd, dda.ALPHA_LDR)
    sweep = [dda.waves_for_orientation(0.4, th, 0.3) for th in (0.6, 0.75, 0.9, 1.05)]
    hist = [[], []]
    for kh, es, _ in sweep[:3]:
        for l in range(2):
            a = dda.site_inverse_polarizability(comp, m, kd, dda.ALPHA_LDR, kh, es[l])
            hist[l].append((dda.solve_dense(r, kd, a, dda.incident_field(r, kd, kh, es[l])), a, kh))
    kn, en, _ = sweep[3]
    expect = []
    for l in range(2):
        an = dda.site_inverse_polarizability(comp, m, kd, dda.ALPHA_LDR, kn, en[l])
        En = dda.incident_field(r, kd, kn, en[l])
        P0, _ = dda.projected_history_guess(r, kd, an, kn, En, hist[l])
        expect.append(np.linalg.norm(En - dda.matvec_direct(r, kd, an, P0)) / np.linalg.norm(En))
    for i, (kh, es, _) in enumerate(sweep[:3]):
        ctx.solve([kh, kh], es, prec=P.DDA_SOLVE_FP64, tol=1e-11, want_p=False, history=3,
                  guess=P.DDA_GUESS_ZERO if i == 0 else P.DDA_GUESS_PREV)
    _, st, _ = ctx.solve([kn, kn], en, prec=P.DDA_SOLVE_FP64, tol=1e-5, guess=P.DDA_GUESS_PROJECT, history=3)
    for l in range(2):
        assert abs(st[l]["guess_resid"] - expect[l]) <= 1e-7 + 1e-5 * expect[l], (l, st[l], expect[l])
        assert st[l]["rel_resid"] <= 1e-5
    with pytest.raises(P.DDAError):
        ctx.solve([kn, kn], en, guess=P.DDA_GUESS_PROJECT, history=5)


def test_zero_guess_shortcut_matches_a_zero_user_guess(ctx):
    """From P0 = 0 the first FP64 residual is E itself, which the solve takes
    without a matvec; a user guess of zeros takes the matvec path (E - A 0).
    Both give E exactly, so solutions and iteration counts are identical, and
    the shortcut saves one matvec per rhs."""
    import paper_1002_1505_amd as P

    occ = synth.ellipsoid_occupancy((12, 10, 9), (11.5, 9.4, 8.6))
    r, comp = _setup(ctx, occ, [1.45 + 0.08j], 0.35, dda.ALPHA_LDR)
    khat, es, L = dda.waves_for_orientation(0.4, 0.8, 0.3)
    for prec in (P.DDA_SOLVE_FP32_REFINE, P.DDA_SOLVE_FP64):
        Pz, sz, _ = ctx.solve([khat, khat], es, prec=prec, tol=1e-6)
        zeros = [np.zeros((len(r), 3), np.complex128) for _ in range(2)]
        Pu, su, _ = ctx.solve([khat, khat], es, prec=prec, tol=1e-6, guess=P.DDA_GUESS_USER, p0=zeros)
        for l in range(2):
            assert sz[l]["iters"] == su[l]["iters"] and sz[l]["outer"] == su[l]["outer"], (prec, l)
            assert sz[l]["matvecs"] == su[l]["matvecs"] - 1, (prec, l)
            assert np.array_equal(Pz[l], Pu[l]), (prec, l)
            assert sz[l]["rel_resid"] == su[l]["rel_resid"] and sz[l]["rel_resid"] <= 1e-6


def test_amplitudes_per_rhs_match_shared_directions_and_oracle(ctx):
    """dda_amplitudes_per_rhs: two orientations x two polarizations, each
    orientation with the scattering directions of its own lab frame (37
    angles in one plane): the same values as dda_amplitudes over the union of
    the directions (each rhs's own block), and the oracle's amplitudes of the
    oracle's FP64 solutions to the solve's tolerance."""
    import paper_1002_1505_amd as P

    occ = synth.ellipsoid_occupancy((12, 10, 9), (11.5, 9.6, 8.4))
    r, comp, _ = dda.sites_from_occupancy(occ)
    m, kd = 1.45 + 0.05j, 0.35
    ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
    th = np.deg2rad(np.arange(0, 181, 5.0))
    ph = np.full_like(th, 0.7)
    kh, ee, frames, Ps_or = [], [], [], []
    for ori in ((0.2, 0.5, 1.0), (1.1, 2.0, 0.3)):
        khat, es, L = dda.waves_for_orientation(*ori)
        n_lab, t_lab, p_lab = scatter.lab_direction_basis(th, ph)
        frames.append((n_lab @ L, np.concatenate([t_lab @ L, p_lab @ L], axis=1), L))
        for e in es:
            kh.append(khat)
            ee.append(e)
            ainv = dda.site_inverse_polarizability(comp, [m], kd, dda.ALPHA_LDR, khat, e)
            Ps_or.append(dda.solve_iterative(r, kd, ainv, dda.incident_field(r, kd, khat, e), tol=1e-11)[0])
    Pg, st, status = ctx.solve(kh, ee, tol=1e-9, prec=P.DDA_SOLVE_FP64)
    assert status == 0
    n_per = np.stack([frames[i // 2][0] for i in range(4)])
    e_per = np.stack([frames[i // 2][1] for i in range(4)])
    f_per = ctx.amplitudes_per_rhs(4, n_per, e_per)
    f_all = ctx.amplitudes(4, np.concatenate([fr[0] for fr in frames]), np.concatenate([fr[1] for fr in frames]))
    nd = len(th)
    for i in range(4):
        own = f_all[i, (i // 2) * nd:(i // 2 + 1) * nd]
        assert np.max(np.abs(f_per[i] - own)) <= 1e-12 * np.max(np.abs(own)), i
    for o in range(2):
        fo = scatter.scattering_amplitudes(r, kd, Ps_or[2 * o:2 * o + 2], th, ph, frames[o][2])  # (dir, m, l)
        fg = np.transpose(f_per[2 * o:2 * o + 2], (1, 2, 0))
        assert np.max(np.abs(fg - fo)) / np.max(np.abs(fo)) < 1e-7, o
    with pytest.raises(P.DDAError):
        ctx.amplitudes_per_rhs(3, n_per[:3], e_per[:3])
