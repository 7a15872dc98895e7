"""Pins of the FP64 reference of the learned initialiser's network.

Convolution against a brute-force loop; exact adjoint identities of every
linear piece; the whole-network wiring against closed forms (weights that
route one channel through chosen layers give block averages of the input);
the whole backward pass against central finite differences."""
import numpy as np
import pytest

from oracle import unet


def _brute_conv(x, w, b):
    bsz, h, wd, _ = x.shape
    y = np.zeros((bsz, h, wd, w.shape[0]))
    for n in range(bsz):
        for i in range(h):
            for j in range(wd):
                for o in range(w.shape[0]):
                    s = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            ii, jj = i + ky - 1, j + kx - 1
                            if 0 <= ii < h and 0 <= jj < wd:
                                s += float(np.dot(x[n, ii, jj], w[o, ky, kx]))
                    y[n, i, j, o] = s
    return y


def test_conv_matches_brute_force():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 5, 6, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(unet.conv(x, w, b), _brute_conv(x, w, b), rtol=0, atol=1e-12)


def test_conv_backward_is_the_adjoint():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 7, 5, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    dy = rng.standard_normal((2, 7, 5, 4))
    dx, dw, db = unet.conv_backward(x, w, dy)
    y0 = unet.conv(x, w, np.zeros(4))
    # <conv(x, w), dy> is bilinear in (x, w): both partial adjoints reproduce it
    ref = float(np.sum(y0 * dy))
    assert abs(float(np.sum(x * dx)) - ref) <= 1e-10 * abs(ref)
    assert abs(float(np.sum(w * dw)) - ref) <= 1e-10 * abs(ref)
    np.testing.assert_allclose(db, dy.sum(axis=(0, 1, 2)), rtol=1e-12)


def test_pool_and_up_adjoints_and_identities():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 8, 6, 3))
    y = rng.standard_normal((2, 4, 3, 3))
    assert abs(np.sum(unet.pool(x) * y) - np.sum(x * unet.pool_backward(y))) <= 1e-12
    z = rng.standard_normal((2, 16, 12, 3))
    assert abs(np.sum(unet.up(x) * z) - np.sum(x * unet.up_backward(z))) <= 1e-10
    np.testing.assert_allclose(unet.pool(unet.up(x)), x, atol=1e-15)
    assert unet.pool(x)[0, 1, 2, 0] == pytest.approx(x[0, 2:4, 4:6, 0].mean(), abs=1e-15)


def _routing_params(select):
    """Weights that copy one input channel to output channel 0 through the
    centre tap; `select[i]` is the input channel layer i reads (None: zero layer)."""
    ps = unet.unflatten(np.zeros(unet.num_params()))
    for i, c in enumerate(select):
        if c is not None:
            ps[2 * i][0, 1, 1, c] = 1.0
    return unet.flatten(ps)


def _blocks(x, f):
    b, h, w = x.shape
    return x.reshape(b, h // f, f, w // f, f).mean(axis=(2, 4))


def _rep(x, f):
    return np.repeat(np.repeat(x, f, axis=1), f, axis=2)


def test_network_wiring_closed_forms():
    rng = np.random.default_rng(4)
    x = rng.uniform(0.0, 1.0, (2, 128, 128, 2))
    x0 = x[..., 0]
    # through the bottleneck: 16 x 16 block means, repeated 8x
    y, _ = unet.forward(_routing_params([0, 0, 0, 0, 0, 0, 0, 0, 0, 0]), x)
    np.testing.assert_allclose(y[..., 0], _rep(_blocks(x0, 16), 8), atol=1e-13)
    assert np.all(y[..., 1] == 0)
    # L8 reads the e1 skip (input channel 64 of 96): 2 x 2 block means
    y, _ = unet.forward(_routing_params([0, 0, None, None, None, None, None, None, 64, 0]), x)
    np.testing.assert_allclose(y[..., 0], _blocks(x0, 2), atol=1e-13)
    # L7 reads the e2 skip (channel 128 of 192), L8 the upsampled path (channel 0)
    y, _ = unet.forward(_routing_params([0, 0, 0, None, None, None, None, 128, 0, 0]), x)
    np.testing.assert_allclose(y[..., 0], _rep(_blocks(x0, 4), 2), atol=1e-13)
    # L6 reads the e3 skip (channel 256 of 384)
    y, _ = unet.forward(_routing_params([0, 0, 0, 0, None, None, 256, 0, 0, 0]), x)
    np.testing.assert_allclose(y[..., 0], _rep(_blocks(x0, 8), 4), atol=1e-13)
    # output channel 1 and the biases
    ps = unet.unflatten(_routing_params([0] * 10))
    ps[19][:] = [0.25, -0.5]
    y, _ = unet.forward(unet.flatten(ps), x)
    np.testing.assert_allclose(y[..., 1], -0.5, atol=0)
    # relu: a negated input is cut at L0
    y, _ = unet.forward(_routing_params([0] * 10), -x)
    assert np.all(y[..., 0] == 0)


def test_parameter_count():
    assert unet.num_params() == sum(9 * ci * co + co for ci, co, _, _ in unet.LAYERS)
    assert 1_000_000 < unet.num_params() < 2_500_000


@pytest.fixture(scope="module")
def fd_setup():
    rng = np.random.default_rng(5)
    flat = unet.init_params(3)
    flat[unet.num_params() - 2:] = [0.3, -0.2]
    x = rng.uniform(0.0, 1.0, (1, 128, 128, 2))
    t = rng.standard_normal((1, 64, 64, 2)) * 0.1
    loss, g = unet.loss_and_grad(flat, x, t)
    return flat, x, t, loss, g


def _layer_mask(i):
    m = np.zeros(unet.num_params())
    off = 0
    for j, s in enumerate(unet.param_shapes()):
        n = int(np.prod(s))
        if j // 2 == i:
            m[off:off + n] = 1
        off += n
    return m


@pytest.mark.parametrize("which", ["all", 0, 3, 5, 6, 8, 9])
def test_network_gradient_finite_differences(fd_setup, which):
    flat, x, t, loss, g = fd_setup
    rng = np.random.default_rng(17 if which == "all" else 100 + which)
    d = rng.standard_normal(flat.size)
    if which != "all":
        d *= _layer_mask(which)
    d /= np.linalg.norm(d)
    h = 1e-6
    lp = unet.loss_and_grad(flat + h * d, x, t)[0]
    lm = unet.loss_and_grad(flat - h * d, x, t)[0]
    fd = (lp - lm) / (2 * h)
    an = float(g @ d)
    assert abs(fd - an) <= 1e-5 * abs(an) + 1e-9 * loss, (fd, an)
