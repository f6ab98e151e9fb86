"""Oracle for the learned initial guess (test infrastructure only).

A plain FP64 numpy version of the small 3D convolutional network the GPU
library trains and runs: 3x3x3 convolutions with zero padding and dilation,
ReLU, a masked squared-error loss, and Adam.  The guide itself has no learned
component; the network is the library's predictor of the Krylov initial
guess (the guide's default guess is P = 0, "Choice of Iterative Algorithm").

Layout: activations are channels-last arrays x[z, y, x, c]; a weight tensor
is w[o, ci, co] with the 27 offsets o = (dz+1)*9 + (dy+1)*3 + (dx+1),
dx, dy, dz in {-1, 0, 1}, and the layer reads x[v + d * offset].
"""
from __future__ import annotations

import numpy as np

OFFSETS = np.array([(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)])


def _shift(x, off, d):
    """x[v + d * off] with zeros outside the box (x: (D, D, D, C))."""
    D = x.shape[:3]
    out = np.zeros_like(x)
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    for a in range(3):
        s = int(off[a]) * d
        if s >= 0:
            src[a] = slice(s, D[a])
            dst[a] = slice(0, D[a] - s)
        else:
            src[a] = slice(0, D[a] + s)
            dst[a] = slice(-s, D[a])
    out[tuple(dst)] = x[tuple(src)]
    return out


def conv3d(x, w, b, d=1):
    """y[v, co] = b[co] + sum_o sum_ci x[v + d off_o, ci] w[o, ci, co]."""
    y = np.zeros(x.shape[:3] + (w.shape[2],))
    for o, off in enumerate(OFFSETS):
        y += _shift(x, off, d) @ w[o]
    return y + b


def conv3d_backward(x, w, dy, d=1):
    """(dx, dw, db) of conv3d for upstream gradient dy."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for o, off in enumerate(OFFSETS):
        xs = _shift(x, off, d)
        dw[o] = xs.reshape(-1, x.shape[3]).T @ dy.reshape(-1, dy.shape[3])
        dx += _shift(dy @ w[o].T, -off, d)
    db = dy.reshape(-1, dy.shape[3]).sum(0)
    return dx, dw, db


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    bfloat16 keeps the 8 high mantissa bits of an IEEE float32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


class Net:
    """Stack of 3x3x3 convolutions; ReLU after every layer but the last.

    layers: list of (cin, cout, dilation).  Parameters: list of (w, b).
    `quantize` (default: none) is applied where a reduced-precision
    implementation stores values: hidden activations after the ReLU, the
    output gradient, and the data gradient of every hidden layer.
    """

    def __init__(self, layers, params, quantize=None):
        self.layers = layers
        self.params = params
        self.q = quantize if quantize is not None else (lambda a: a)

    def forward(self, x):
        acts = [x]
        h = x
        for i, ((cin, cout, d), (w, b)) in enumerate(zip(self.layers, self.params)):
            h = conv3d(h, w, b, d)
            if i < len(self.layers) - 1:
                h = self.q(np.maximum(h, 0.0))
            acts.append(h)
        return h, acts

    def backward(self, acts, dout):
        grads = [None] * len(self.layers)
        g = self.q(dout)
        for i in range(len(self.layers) - 1, -1, -1):
            cin, cout, d = self.layers[i]
            w, b = self.params[i]
            dx, dw, db = conv3d_backward(acts[i], w, g, d)
            grads[i] = (dw, db)
            if i > 0:
                g = self.q(dx * (acts[i] > 0))
        return grads


def masked_mse(out, target, mask, nout):
    """Loss = sum over masked voxels of |out[..., :nout] - target|^2 / (sum |target|^2);
    returns (loss, d loss / d out)."""
    m = mask[..., None].astype(np.float64)
    diff = (out[..., :nout] - target) * m
    den = float(np.sum((target * m) ** 2))
    loss = float(np.sum(diff ** 2)) / den
    dout = np.zeros_like(out)
    dout[..., :nout] = 2.0 * diff / den
    return loss, dout


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One Adam update (Kingma & Ba 2015) with decoupled weight decay; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v
