"""Failure handling of the solve on the GPU, every condition forced from the
host so that every kernel still ends normally: an iteration budget that is
too small, |m| k d >= 1, the breakdown restart of the inner BiCGstab (forced
by the restart_every test hook of the solve options), guesses and fields
that are not finite, a polarization vector that is not a unit vector, the
per-iteration residual trace (DDA_TRACE) and the network's save/load round
trip.  Expected values come from the oracle (residuals) or from the
library's own unforced solve of the same system (restarts change the
iterates, not the solution)."""
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


def _target(ctx, n=12, m=1.5 + 0.1j, kd=0.4):
    import paper_1002_1505_amd as P

    occ = synth.sphere_occupancy(n)
    ctx.set_target(occ, [m], kd, P.DDA_ALPHA_LDR)
    r, comp, _ = dda.sites_from_occupancy(occ)
    return r, comp


def test_small_iteration_budget_warns_not_converged(ctx):
    import paper_1002_1505_amd as P

    r, comp = _target(ctx)
    kh, es, _ = dda.waves_for_orientation(0.2, 0.5, 0.1)
    for prec in (P.DDA_SOLVE_FP32_REFINE, P.DDA_SOLVE_FP64):
        print(f"max_iter=3 prec={prec}", flush=True)
        Pg, st, status = ctx.solve([kh, kh], es, tol=1e-8, max_iter=3, prec=prec)
        assert status == P.DDA_WARN_NOT_CONVERGED
        for l in range(2):
            assert st[l]["status"] == P.DDA_WARN_NOT_CONVERGED
            assert st[l]["iters"] <= 3
            assert np.all(np.isfinite(Pg[l]))
            # the reported residual is the true FP64 residual of the returned P
            ainv = dda.site_inverse_polarizability(comp, [1.5 + 0.1j], 0.4, dda.ALPHA_LDR, kh, es[l])
            rel, _ = dda.residual_norms(r, 0.4, ainv, dda.incident_field(r, 0.4, kh, es[l]), Pg[l])
            assert 1e-8 < rel < 1.0 and abs(rel - st[l]["rel_resid"]) <= 1e-9 + 1e-6 * rel


def test_mkd_at_least_one_warns_and_still_solves(ctx):
    import paper_1002_1505_amd as P

    occ = synth.sphere_occupancy(8)
    st = ctx.set_target(occ, [2.5 + 0.1j], 0.45, P.DDA_ALPHA_LDR)  # |m| k d = 1.126
    assert st == P.DDA_WARN_MKD_GE_1
    assert "m" in ctx.last_error()
    st = ctx.set_target(occ, [1.5 + 0.1j], 0.45, P.DDA_ALPHA_LDR)  # 0.677: no warning
    assert st == 0
    ctx.set_target(occ, [2.5 + 0.1j], 0.45, P.DDA_ALPHA_LDR)
    kh, es, _ = dda.waves_for_orientation(0.0, 0.3, 0.0)
    _, s, status = ctx.solve([kh, kh], es, want_p=False, max_iter=5000)
    assert status == 0 and all(x["rel_resid"] <= 1e-5 for x in s)


@pytest.mark.parametrize("prec_name", ["fp32_refine", "fp64"])
@pytest.mark.parametrize("graph", [True, False])
def test_forced_restarts_reach_the_same_solution(ctx, prec_name, graph):
    """restart_every = k sets the breakdown flag after every k-th iteration,
    so the restart branch of the update, scalar and flush kernels runs
    (rhat = p = r, rho = ||r||^2): the solve still reaches tol with the same
    solution, in at least as many iterations."""
    import paper_1002_1505_amd as P

    r, comp = _target(ctx, n=16, m=1.6 + 0.05j, kd=0.45)
    kh, es, _ = dda.waves_for_orientation(0.7, 1.1, 0.4)
    prec = P.DDA_SOLVE_FP64 if prec_name == "fp64" else P.DDA_SOLVE_FP32_REFINE
    flags = 0 if graph else P.DDA_NO_GRAPH
    ref, sref, _ = ctx.solve([kh, kh], es, tol=1e-7, prec=prec, flags=flags)
    for k in (1, 3):
        print(f"restart_every={k} prec={prec_name} graph={graph}", flush=True)
        Pr, sr, status = ctx.solve([kh, kh], es, tol=1e-7, prec=prec, flags=flags, restart_every=k, max_iter=5000)
        assert status == 0
        for l in range(2):
            assert sr[l]["rel_resid"] <= 1e-7
            assert sr[l]["iters"] >= sref[l]["iters"]
            d = np.abs(Pr[l] - ref[l])
            assert np.linalg.norm(d) <= 5e-6 * np.linalg.norm(ref[l])
            assert d.max() <= 5e-5 * np.abs(ref[l]).max()  # every element, not only the norm
    # restart after every iteration is steepest descent on the BiCGstab
    # polynomial: it must be slower than the unforced solve
    assert sum(s["iters"] for s in sr) > sum(s["iters"] for s in sref)
    with pytest.raises(P.DDAError):
        ctx.solve([kh, kh], es, restart_every=-1, want_p=False)


def test_non_finite_guess_falls_back_to_zero(ctx):
    import paper_1002_1505_amd as P

    r, comp = _target(ctx)
    kh, es, _ = dda.waves_for_orientation(0.0, 0.2, 0.0)
    bad = [np.full((len(r), 3), np.nan + 0j), np.full((len(r), 3), np.inf + 0j)]
    bad[1][1:] = 0.1
    for prec in (P.DDA_SOLVE_FP32_REFINE, P.DDA_SOLVE_FP64):
        Pg, st, status = ctx.solve([kh, kh], es, prec=prec, guess=P.DDA_GUESS_USER, p0=bad)
        assert status == 0
        for l in range(2):
            assert st[l]["guess_resid"] == 1.0 and st[l]["rel_resid"] <= 1e-5
            assert np.all(np.isfinite(Pg[l]))


def test_non_finite_field_and_non_unit_polarization_are_rejected(ctx):
    import paper_1002_1505_amd as P

    r, comp = _target(ctx)
    kh, es, _ = dda.waves_for_orientation(0.0, 0.2, 0.0)
    E = [dda.incident_field(r, 0.4, kh, e) for e in es]
    E[1] = E[1].copy()
    E[1][5, 2] = np.nan
    with pytest.raises(P.DDAError) as ei:
        ctx.solve([kh, kh], es, e_inc=E)
    assert ei.value.status == -1
    with pytest.raises(P.DDAError) as ei:
        ctx.solve([kh, kh], [2 * es[0], es[1]], want_p=False)
    assert ei.value.status == -1
    # the context is still usable
    _, st, status = ctx.solve([kh, kh], es, want_p=False)
    assert status == 0


def test_trace_records_every_iteration(ctx, tmp_path):
    """DDA_TRACE appends the FP64 residual checks and the per-iteration
    residual estimates of each solve: the last FP64 line of each rhs is the
    reported residual, the inner lines count the reported iterations."""
    import paper_1002_1505_amd as P

    _target(ctx)
    kh, es, _ = dda.waves_for_orientation(0.3, 0.6, 0.9)
    path = tmp_path / "trace.txt"
    os.environ["DDA_TRACE"] = str(path)
    try:
        _, st, _ = ctx.solve([kh, kh], es, tol=1e-6, want_p=False, prec=P.DDA_SOLVE_FP32_REFINE)
    finally:
        del os.environ["DDA_TRACE"]
    lines = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for i in range(2):
        fp = [float(l[3]) for l in lines if int(l[0]) == i and l[4] == "fp64"]
        inner = [float(l[3]) for l in lines if int(l[0]) == i and l[4] == "inner"]
        assert fp[0] == 1.0 and fp[-1] == pytest.approx(st[i]["rel_resid"], rel=1e-6)
        assert len(fp) == st[i]["outer"]
        assert len(inner) == st[i]["iters"]
        assert inner[-1] < 1e-3 * inner[0]
    # no trace once the variable is unset
    _, st, _ = ctx.solve([kh, kh], es, tol=1e-6, want_p=False)
    assert sum(1 for l in open(path) if l.strip() and not l.startswith("#")) == len(lines)


def test_network_save_load_round_trip(ctx, tmp_path):
    import paper_1002_1505_amd as P

    a = P.Net(ctx, width=16, depth=4, seed=3)
    b = P.Net(ctx, width=16, depth=4, seed=4)
    c = P.Net(ctx, width=32, depth=4, seed=4)
    try:
        rng = np.random.default_rng(0)
        pa = [(rng.standard_normal(w.shape).astype(np.float32), rng.standard_normal(bb.shape).astype(np.float32))
              for w, bb in a.get_params()]
        flat = lambda ps: np.concatenate([np.concatenate([w.reshape(-1), bb.reshape(-1)]) for w, bb in ps])
        a.set_params(pa)
        path = str(tmp_path / "net.bin")
        a.save(path)
        assert not np.array_equal(flat(b.get_params()), flat(pa))
        b.load(path)
        assert np.array_equal(flat(b.get_params()), flat(pa))
        with pytest.raises(P.DDAError):  # another architecture
            c.load(path)
        with pytest.raises(P.DDAError):  # no such file
            b.load(str(tmp_path / "missing.bin"))
        assert np.array_equal(flat(b.get_params()), flat(pa))
    finally:
        for n in (a, b, c):
            n.close()
