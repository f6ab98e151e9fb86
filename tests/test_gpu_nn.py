"""The learned-guess network on the GPU (BF16 MFMA kernels, FP32 accumulate)
against the FP64 oracle network: forward output and parameter gradients.

Weights and inputs are rounded to BF16 before both sides see them.  Two
comparisons: (1) against the oracle that rounds activations and gradients to
BF16 at the same points as the kernels (same rounding decisions; what
remains is FP32-vs-FP64 accumulation order and the occasional BF16 tie that
falls the other way) -- 1 % relative L2, cosine >= 0.9999; (2) against the
pure FP64 oracle, where BF16 rounding (2^-9 relative per store) compounds
over the layers -- 5 % relative L2, cosine >= 0.998."""
import numpy as np
import pytest

from oracle import nn as onn

pytestmark = pytest.mark.gpu


def bf16(a):
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("width,depth,D", [(16, 3, 16), (32, 4, 16), (64, 3, 16), (16, 4, 32)])
def test_forward_and_gradients_match_oracle(width, depth, D):
    """Width 64 runs the channel-split convolution (four 16-channel output
    slices per voxel block) and the weight gradient in four tile groups; the
    32^3 box runs rows of two 16-voxel groups and the dilated layers' shifted
    output-gradient copies with more of each row inside the box."""
    import paper_1002_1505_amd as P

    ctx = P.Context(0)
    net = P.Net(ctx, width=width, depth=depth, seed=3)
    rng = np.random.default_rng(width + depth)
    layers = net.layers()
    params = []
    for cin, cout, d in layers:
        params.append((bf16(rng.standard_normal((27, cin, cout)) * np.sqrt(2.0 / (27 * cin))),
                       (rng.standard_normal(cout) * 0.05).astype(np.float32)))
    net.set_params(params)
    ns = 2
    x = bf16(rng.standard_normal((ns, D, D, D, 16)))
    mask = rng.random((ns, D, D, D)) < 0.4
    target = rng.standard_normal((ns, D, D, D, 16)).astype(np.float32)
    out, grads, loss = net.forward_backward(x, target, mask, nout=6)
    for quant, tol, cmin in ((onn.bf16_round, 1e-2, 0.9999), (None, 5e-2, 0.998)):
        onet = onn.Net(layers, [(w.astype(np.float64), b.astype(np.float64)) for w, b in params], quantize=quant)
        losses, ograds = [], None
        for s in range(ns):
            o, acts = onet.forward(x[s].astype(np.float64))
            rel = np.linalg.norm(out[s] - o) / np.linalg.norm(o)
            assert rel < tol, (quant, rel)
            ls, dout = onn.masked_mse(o, target[s][..., :6].astype(np.float64), mask[s], 6)
            losses.append(ls)
            g = onet.backward(acts, dout / ns)
            ograds = g if ograds is None else [(a[0] + b[0], a[1] + b[1]) for a, b in zip(ograds, g)]
        assert abs(loss - np.mean(losses)) / np.mean(losses) < tol
        for li, ((gw, gb), (ow, ob)) in enumerate(zip(grads, ograds)):
            rel = np.linalg.norm(gw - ow) / np.linalg.norm(ow)
            cos = np.sum(gw * ow) / (np.linalg.norm(gw) * np.linalg.norm(ow))
            assert rel < tol and cos > cmin, (quant, li, rel, cos)
            relb = np.linalg.norm(gb - ob) / np.linalg.norm(ob)
            assert relb < tol, (quant, li, relb)
    net.close()
    ctx.close()


def _sweep_waves(count, beta=0.3, phi=0.2):
    import synth
    from oracle import dda

    out = []
    for b, th, ph in synth.theta_sweep(count, beta, phi):
        kh, es, _ = dda.waves_for_orientation(b, th, ph)
        out.append(([kh, kh], es))
    return out


def test_zero_network_reproduces_projected_guess_and_state_errors():
    """The network starts with a zero last layer, so its guess is the
    least-squares guess it corrects; the learned guess needs a previous
    solution and recording needs a PROJECT or NN solve."""
    import synth
    import paper_1002_1505_amd as P

    ctx = P.Context(0)
    ctx.set_target(synth.sphere_occupancy(16), [1.5 + 0.05j], 0.6, P.DDA_ALPHA_LDR)
    net = P.Net(ctx, width=16, depth=4, seed=5)
    net.attach()
    sw = _sweep_waves(6)
    with pytest.raises(P.DDAError):
        ctx.solve(*sw[0], guess=P.DDA_GUESS_NN, want_p=False)
    ctx.solve(*sw[0], prec=P.DDA_SOLVE_FP64, tol=1e-10, want_p=False)
    ctx.solve(*sw[1], prec=P.DDA_SOLVE_FP64, tol=1e-10, want_p=False, guess=P.DDA_GUESS_PREV_SHIFT)
    with pytest.raises(P.DDAError):
        net.record()
    res = {}
    for name, g in (("project", P.DDA_GUESS_PROJECT), ("nn", P.DDA_GUESS_NN)):
        for hist in (0, 2):
            ctx.solve(*sw[0], prec=P.DDA_SOLVE_FP64, tol=1e-10, want_p=False, history=hist)
            ctx.solve(*sw[1], prec=P.DDA_SOLVE_FP64, tol=1e-10, want_p=False, history=hist,
                      guess=P.DDA_GUESS_PREV)
            _, st, _ = ctx.solve(*sw[2], prec=P.DDA_SOLVE_FP64, tol=1e-5, guess=g, want_p=False, history=hist)
            res[name, hist] = [s["guess_resid"] for s in st]
            assert all(s["rel_resid"] <= 1e-5 for s in st)
    for hist in (0, 2):
        for a, b in zip(res["nn", hist], res["project", hist]):
            assert a < 1.0 and abs(a - b) <= 1e-5 * b + 1e-7, (hist, a, b)
    # two earlier solutions span a better guess than the previous one alone
    assert sum(res["project", 2]) < sum(res["project", 0])
    net.record()
    assert net.num_samples == 2
    net.close()
    ctx.close()


def test_training_lowers_guess_residual_on_its_sweep():
    """Record the solutions of a 12-orientation sweep of a porous aggregate
    (least-squares guesses over a history of 2), train, then run the sweep
    again: the learned guess starts closer to the solution than the
    least-squares guess it corrects."""
    import synth
    import paper_1002_1505_amd as P

    ctx = P.Context(0)
    occ = synth.aggregate_occupancy(16, np.random.default_rng(synth.CONFIG_SEED_BASE + 50))
    ctx.set_target(occ, [1.5 + 0.05j], 0.8, P.DDA_ALPHA_LDR)
    net = P.Net(ctx, width=16, depth=4, seed=7)
    sw = _sweep_waves(12)
    ctx.solve(*sw[0], want_p=False, history=2)
    for w in sw[1:]:
        ctx.solve(*w, guess=P.DDA_GUESS_PROJECT, want_p=False, history=2)
        net.record()
    assert net.num_samples == 22
    first = net.train(epochs=1, batch=2, lr=2e-3)
    last = net.train(epochs=60, batch=2, lr=2e-3)
    assert last < 0.8 * first, (first, last)
    net.attach()
    res = {}
    for name, g in (("project", P.DDA_GUESS_PROJECT), ("nn", P.DDA_GUESS_NN)):
        ctx.solve(*sw[0], want_p=False, history=2)
        r = []
        for w in sw[1:]:
            _, st, _ = ctx.solve(*w, guess=g, want_p=False, history=2)
            assert all(s["rel_resid"] <= 1e-5 for s in st)
            r += [s["guess_resid"] for s in st]
        res[name] = np.mean(r)
    assert res["nn"] < res["project"], res
    net.close()
    ctx.close()


def test_profile_hook_counts_flops_and_times():
    """The timing hook reports positive times and the dense forward FLOP count
    2 x 27 x cin x cout x D^3 x samples summed over the layers."""
    import paper_1002_1505_amd as P

    ctx = P.Context(0)
    net = P.Net(ctx, width=16, depth=4, seed=2)
    f_ms, b_ms, gflop = net.profile(32, 2, 2)
    expect = sum(2.0 * 27 * cin * cout * 32 ** 3 * 2 for cin, cout, _ in net.layers()) * 1e-9
    assert f_ms > 0 and b_ms > 0 and abs(gflop - expect) < 1e-9 * expect
    with pytest.raises(P.DDAError):
        net.profile(24, 2, 1)  # box side not a multiple of 16
    net.close()
    ctx.close()


def test_million_parameter_network_builds_and_runs():
    """The learned-guess network at its full size: width 64, depth 10 holds
    27 (16 x 64 + 8 x 64 x 64 + 64 x 16) weights and 9 x 64 + 16 biases
    (940,624 parameters); its forward and backward passes run on a 64^3 box.
    Widths other than 16, 32 and 64 are refused."""
    import paper_1002_1505_amd as P
    from paper_1002_1505_amd import _lib as L

    ctx = P.Context(0)
    net = P.Net(ctx, width=64, depth=10, seed=4)
    assert net.num_params == 27 * (16 * 64 + 8 * 64 * 64 + 64 * 16) + 9 * 64 + 16
    assert [l[:2] for l in net.layers()] == [(16, 64)] + [(64, 64)] * 8 + [(64, 16)]
    f_ms, b_ms, gflop = net.profile(64, 2, 1)
    print(f"[width 64 depth 10] forward {f_ms:.3f} ms backward {b_ms:.3f} ms for 2 samples of 64^3, "
          f"{gflop / f_ms:.1f} TFLOP/s forward", flush=True)
    assert f_ms > 0 and b_ms > 0
    net.close()
    with pytest.raises(P.DDAError) as e:
        P.Net(ctx, width=48, depth=4, seed=1)
    assert e.value.status == L.DDA_ERR_INVALID_ARG
    ctx.close()


def test_save_load_round_trip(tmp_path):
    """dda_nn_save / dda_nn_load: a network loaded into a fresh one (other
    seed) holds the same parameters bit for bit and gives the same forward
    output bit for bit; a file of another shape, a truncated file and a
    missing file are refused with the documented status."""
    import paper_1002_1505_amd as P
    from paper_1002_1505_amd import _lib as L

    ctx = P.Context(0)
    a = P.Net(ctx, width=16, depth=3, seed=3)
    rng = np.random.default_rng(11)
    params = [(bf16(rng.standard_normal((27, cin, cout)) * 0.1), (rng.standard_normal(cout) * 0.05).astype(np.float32))
              for cin, cout, _ in a.layers()]
    a.set_params(params)
    x = bf16(rng.standard_normal((1, 16, 16, 16, 16)))
    out_a, _, _ = a.forward_backward(x)
    path = str(tmp_path / "net.bin")
    a.save(path)
    b = P.Net(ctx, width=16, depth=3, seed=9)
    assert not all(np.array_equal(p[0], q[0]) for p, q in zip(b.get_params(), a.get_params()))
    b.load(path)
    for (wa, ba), (wb, bb) in zip(a.get_params(), b.get_params()):
        assert np.array_equal(wa, wb) and np.array_equal(ba, bb)
    out_b, _, _ = b.forward_backward(x)
    assert np.array_equal(out_a, out_b)
    other = P.Net(ctx, width=32, depth=3, seed=3)
    with pytest.raises(P.DDAError) as e:
        other.load(path)
    assert e.value.status == L.DDA_ERR_INVALID_ARG
    raw = open(path, "rb").read()
    short = str(tmp_path / "short.bin")
    open(short, "wb").write(raw[: len(raw) // 2])
    with pytest.raises(P.DDAError) as e:
        b.load(short)
    assert e.value.status == L.DDA_ERR_IO
    with pytest.raises(P.DDAError) as e:
        b.load(str(tmp_path / "missing.bin"))
    assert e.value.status == L.DDA_ERR_IO
    # a refused load leaves the parameters as they were
    for (wa, ba), (wb, bb) in zip(a.get_params(), b.get_params()):
        assert np.array_equal(wa, wb) and np.array_equal(ba, bb)
    for n in (a, b, other):
        n.close()
    ctx.close()
