"""The learned-guess network on the GPU (BF16 MFMA kernels, FP32 accumulate)
against the FP64 oracle network: forward output and parameter gradients.

Weights and inputs are rounded to BF16 before both sides see them, so the
remaining difference comes from the BF16 rounding of the activations and of
the output gradient between layers (8-bit mantissa: ~0.4 % per rounding,
a few roundings deep) -- bars: 3 % relative L2 and cosine >= 0.999."""
import numpy as np
import pytest

from oracle import nn as onn

pytestmark = pytest.mark.gpu


def bf16(a):
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("width,depth", [(16, 3), (32, 4)])
def test_forward_and_gradients_match_oracle(width, depth):
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
    D, ns = 16, 2
    x = bf16(rng.standard_normal((ns, D, D, D, 16)))
    mask = rng.random((ns, D, D, D)) < 0.4
    target = rng.standard_normal((ns, D, D, D, 16)).astype(np.float32)
    out, grads, loss = net.forward_backward(x, target, mask, nout=6)
    onet = onn.Net(layers, [(w.astype(np.float64), b.astype(np.float64)) for w, b in params])
    losses, ograds = [], None
    for s in range(ns):
        o, acts = onet.forward(x[s].astype(np.float64))
        rel = np.linalg.norm(out[s] - o) / np.linalg.norm(o)
        assert rel < 3e-2, rel
        ls, dout = onn.masked_mse(o, target[s].astype(np.float64), mask[s], 6)
        losses.append(ls)
        g = onet.backward(acts, dout / ns)
        ograds = g if ograds is None else [(a[0] + b[0], a[1] + b[1]) for a, b in zip(ograds, g)]
    assert abs(loss - np.mean(losses)) / np.mean(losses) < 2e-2
    for li, ((gw, gb), (ow, ob)) in enumerate(zip(grads, ograds)):
        rel = np.linalg.norm(gw - ow) / np.linalg.norm(ow)
        cos = np.sum(gw * ow) / (np.linalg.norm(gw) * np.linalg.norm(ow))
        assert rel < 3e-2 and cos > 0.999, (li, rel, cos)
        relb = np.linalg.norm(gb - ob) / np.linalg.norm(ob)
        assert relb < 3e-2, (li, relb)
    net.close()
    ctx.close()
