"""FP64 reference of the learned initialiser's network (test infrastructure).

A small U-Net maps the real-space estimate of one window's object patch
(128 x 128, two channels: real and imaginary part; see seed.network_input) to
the amplitude and phase of the central 64 x 64 object patch under the probe.  The layer list (NHWC activations, 3 x 3 convolutions with
zero padding 1 and stride 1, 2 x 2 average pooling, 2x nearest upsampling,
skip connections concatenated after the upsampled channels):

    L0 conv  2 ->  32 @128 relu;  pool -> 64
    L1 conv 32 ->  32 @64  relu  (e1);  pool -> 32
    L2 conv 32 ->  64 @32  relu  (e2);  pool -> 16
    L3 conv 64 -> 128 @16  relu  (e3);  pool -> 8
    L4 conv 128 -> 256 @8  relu
    L5 conv 256 -> 256 @8  relu;  up -> 16, concat e3 (384 ch)
    L6 conv 384 -> 128 @16 relu;  up -> 32, concat e2 (192 ch)
    L7 conv 192 ->  64 @32 relu;  up -> 64, concat e1 (96 ch)
    L8 conv 96 ->  32 @64  relu
    L9 conv 32 ->   2 @64  (linear): channel 0 amplitude, channel 1 phase

Parameters are flattened layer by layer: weights W[cout][ky][kx][cin], then
biases b[cout].  Loss: mean squared error over all outputs.

Everything here is a direct definition (im2col + matmul for the convolution)
with a hand-written backward pass; the tests pin it with central finite
differences.
"""
from __future__ import annotations

import numpy as np

# (cin, cout, size, relu) of L0..L9
LAYERS = [
    (2, 32, 128, True),
    (32, 32, 64, True),
    (32, 64, 32, True),
    (64, 128, 16, True),
    (128, 256, 8, True),
    (256, 256, 8, True),
    (384, 128, 16, True),
    (192, 64, 32, True),
    (96, 32, 64, True),
    (32, 2, 64, False),
]


def param_shapes():
    out = []
    for cin, cout, _, _ in LAYERS:
        out.append((cout, 3, 3, cin))
        out.append((cout,))
    return out


def num_params() -> int:
    return int(sum(np.prod(s) for s in param_shapes()))


def unflatten(flat):
    flat = np.asarray(flat, dtype=np.float64)
    ps, off = [], 0
    for s in param_shapes():
        n = int(np.prod(s))
        ps.append(flat[off:off + n].reshape(s))
        off += n
    assert off == flat.size
    return ps


def flatten(ps):
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in ps])


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / (9 cin))), zero biases."""
    rng = np.random.default_rng([7, seed])
    ps = []
    for cin, cout, _, _ in LAYERS:
        ps.append(rng.standard_normal((cout, 3, 3, cin)) * np.sqrt(2.0 / (9 * cin)))
        ps.append(np.zeros(cout))
    return flatten(ps)


def _im2col(x):
    """(B, H, W, C) -> (B, H, W, 3, 3, C) with zero padding 1."""
    b, h, w, c = x.shape
    xp = np.zeros((b, h + 2, w + 2, c))
    xp[:, 1:-1, 1:-1] = x
    cols = np.empty((b, h, w, 3, 3, c))
    for ky in range(3):
        for kx in range(3):
            cols[:, :, :, ky, kx] = xp[:, ky:ky + h, kx:kx + w]
    return cols


def conv(x, w, bias):
    """y[b,y,x,o] = bias[o] + sum_{ky,kx,c} x[b, y+ky-1, x+kx-1, c] w[o,ky,kx,c]."""
    cols = _im2col(x)
    b, h, ww = x.shape[:3]
    y = cols.reshape(b * h * ww, -1) @ w.reshape(w.shape[0], -1).T + bias
    return y.reshape(b, h, ww, -1)


def conv_backward(x, w, dy):
    """(dx, dw, db) of conv for the upstream gradient dy."""
    b, h, ww, cin = x.shape
    cout = w.shape[0]
    cols = _im2col(x).reshape(b * h * ww, 9 * cin)
    d2 = dy.reshape(b * h * ww, cout)
    dw = (d2.T @ cols).reshape(w.shape)
    db = d2.sum(axis=0)
    dcols = (d2 @ w.reshape(cout, -1)).reshape(b, h, ww, 3, 3, cin)
    dxp = np.zeros((b, h + 2, ww + 2, cin))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + h, kx:kx + ww] += dcols[:, :, :, ky, kx]
    return dxp[:, 1:-1, 1:-1], dw, db


def pool(x):
    b, h, w, c = x.shape
    return x.reshape(b, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def pool_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(dy):
    b, h, w, c = dy.shape
    return dy.reshape(b, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def forward(flat, x):
    """Network output (B, 64, 64, 2) for input x (B, 128, 128, 2), plus the cache."""
    ps = unflatten(flat)
    W = ps[0::2]
    Bs = ps[1::2]
    cache = {}

    def layer(i, inp):
        z = conv(inp, W[i], Bs[i])
        a = np.maximum(z, 0.0) if LAYERS[i][3] else z
        cache[i] = (inp, a)
        return a

    a0 = layer(0, x)
    e1 = layer(1, pool(a0))
    e2 = layer(2, pool(e1))
    e3 = layer(3, pool(e2))
    a4 = layer(4, pool(e3))
    a5 = layer(5, a4)
    a6 = layer(6, np.concatenate([up(a5), e3], axis=-1))
    a7 = layer(7, np.concatenate([up(a6), e2], axis=-1))
    a8 = layer(8, np.concatenate([up(a7), e1], axis=-1))
    y = layer(9, a8)
    return y, cache


def backward(flat, cache, dy):
    """Gradient of the loss with respect to the flat parameters, given dL/dy."""
    ps = unflatten(flat)
    W = ps[0::2]
    grads = [None] * len(ps)

    def layer_back(i, da):
        inp, a = cache[i]
        dz = da * (a > 0) if LAYERS[i][3] else da
        dx, dw, db = conv_backward(inp, W[i], dz)
        grads[2 * i], grads[2 * i + 1] = dw, db
        return dx

    d8 = layer_back(9, dy)
    dc8 = layer_back(8, d8)
    d7 = up_backward(dc8[..., :64])
    de1 = dc8[..., 64:]
    dc7 = layer_back(7, d7)
    d6 = up_backward(dc7[..., :128])
    de2 = dc7[..., 128:]
    dc6 = layer_back(6, d6)
    d5 = up_backward(dc6[..., :256])
    de3 = dc6[..., 256:]
    d4 = layer_back(5, d5)
    dp3 = layer_back(4, d4)
    de3 = de3 + pool_backward(dp3)
    dp2 = layer_back(3, de3)
    de2 = de2 + pool_backward(dp2)
    dp1 = layer_back(2, de2)
    de1 = de1 + pool_backward(dp1)
    dp0 = layer_back(1, de1)
    layer_back(0, pool_backward(dp0))
    return flatten(grads)


def loss_and_grad(flat, x, target):
    """(mean squared error, flat gradient)."""
    y, cache = forward(flat, x)
    diff = y - target
    loss = float(np.mean(diff ** 2))
    return loss, backward(flat, cache, 2.0 * diff / diff.size)
