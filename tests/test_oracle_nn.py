"""Pins for the oracle of the learned-guess network: the convolution equals an
independent library correlation, and the backward pass matches finite
differences of the forward pass."""
import numpy as np
from scipy import ndimage

from oracle import nn


def _rand_net(rng, layers):
    params = []
    for cin, cout, d in layers:
        params.append((rng.standard_normal((27, cin, cout)) * 0.3, rng.standard_normal(cout) * 0.1))
    return nn.Net(layers, params)


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    D, cin, cout = 7, 3, 2
    x = rng.standard_normal((D, D, D, cin))
    w = rng.standard_normal((27, cin, cout))
    b = rng.standard_normal(cout)
    for d in (1, 2):
        y = nn.conv3d(x, w, b, d)
        for co in range(cout):
            ref = np.full((D, D, D), b[co])
            for ci in range(cin):
                k = np.zeros((2 * d + 1,) * 3)
                for o, (dz, dy, dx) in enumerate(nn.OFFSETS):
                    k[d * dz + d, d * dy + d, d * dx + d] = w[o, ci, co]
                ref += ndimage.correlate(x[..., ci], k, mode="constant", cval=0.0)
            assert np.allclose(y[..., co], ref, atol=1e-12)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    layers = [(2, 3, 1), (3, 3, 2), (3, 2, 1)]
    net = _rand_net(rng, layers)
    D = 5
    x = rng.standard_normal((D, D, D, 2))
    mask = rng.random((D, D, D)) < 0.6
    target = rng.standard_normal((D, D, D, 2))

    def loss_of(net):
        out, _ = net.forward(x)
        return nn.masked_mse(out, target, mask, 2)[0]

    out, acts = net.forward(x)
    loss, dout = nn.masked_mse(out, target, mask, 2)
    grads = net.backward(acts, dout)
    eps = 1e-6
    for li in range(len(layers)):
        w, b = net.params[li]
        for idx in [(0, 0, 0), (13, 1, 1), (26, -1, -1)]:
            wp = w.copy()
            wp[idx] += eps
            wm = w.copy()
            wm[idx] -= eps
            net.params[li] = (wp, b)
            lp = loss_of(net)
            net.params[li] = (wm, b)
            lm = loss_of(net)
            net.params[li] = (w, b)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - grads[li][0][idx]) <= 1e-6 + 1e-5 * abs(fd), (li, idx)
        bp = b.copy()
        bp[0] += eps
        bm = b.copy()
        bm[0] -= eps
        net.params[li] = (w, bp)
        lp = loss_of(net)
        net.params[li] = (w, bm)
        lm = loss_of(net)
        net.params[li] = (w, b)
        assert abs((lp - lm) / (2 * eps) - grads[li][1][0]) <= 1e-6


def test_adam_matches_textbook_first_step():
    """After one step Adam moves every parameter by -lr * sign(g) (bias-corrected
    moments reduce to g and g^2), up to eps."""
    rng = np.random.default_rng(2)
    p = rng.standard_normal(10)
    g = rng.standard_normal(10)
    p1, m, v = nn.adam_step(p, g, np.zeros(10), np.zeros(10), 1, lr=1e-2)
    assert np.allclose(p1 - p, -1e-2 * np.sign(g), atol=1e-9)


def test_bf16_rounding_known_values():
    """bfloat16 keeps 8 mantissa bits: 1 + 2^-8 rounds to even (1), 1 + 3*2^-8
    rounds up to 1 + 2^-6... checked against exact binary expansions."""
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -2.5, 3.140625])
    r = nn.bf16_round(v)
    assert np.array_equal(r, [1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -2.5, 3.140625])


def test_quantized_backward_equals_plain_backward_without_rounding():
    """With the identity quantizer the two backward formulations agree."""
    rng = np.random.default_rng(4)
    layers = [(2, 3, 1), (3, 2, 2)]
    net = _rand_net(rng, layers)
    x = rng.standard_normal((4, 4, 4, 2))
    out, acts = net.forward(x)
    g = net.backward(acts, np.ones_like(out))
    net2 = nn.Net(layers, net.params, quantize=lambda a: a)
    out2, acts2 = net2.forward(x)
    g2 = net2.backward(acts2, np.ones_like(out2))
    for (a, b), (c, d) in zip(g, g2):
        assert np.allclose(a, c) and np.allclose(b, d)
