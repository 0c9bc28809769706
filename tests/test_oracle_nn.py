"""Pins of the surrogate network's oracle (oracle/nn_oracle.py) against what
the mathematics fixes: scipy's 2-D correlation for the convolution, central
finite differences for every gradient, adjointness of the pooling and
upsampling gradients, closed forms of the loss and of Adam's steps."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import nn_oracle as nn

RNG = np.random.default_rng(7)


def test_conv3x3_matches_scipy_correlation():
    x = RNG.standard_normal((2, 7, 9, 3))
    w = RNG.standard_normal((4, 3, 3, 3))
    b = RNG.standard_normal(4)
    y = nn.conv3x3(x, w, b)
    for bi in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[bi, :, :, c], w[o, :, :, c], mode="same", boundary="fill")
                             for c in range(3))
            assert np.abs(y[bi, :, :, o] - ref).max() < 1e-12


def test_conv_gradients_by_adjointness_and_finite_differences():
    x = RNG.standard_normal((2, 5, 6, 3))
    w = RNG.standard_normal((4, 3, 3, 3))
    dy = RNG.standard_normal((2, 5, 6, 4))
    # <conv(x, w), dy> = <x, dgrad(dy, w)> = <w, wgrad(x, dy)>
    lhs = np.sum(nn.conv3x3(x, w) * dy)
    assert abs(lhs - np.sum(x * nn.conv3x3_dgrad(dy, w))) < 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(w * nn.conv3x3_wgrad(x, dy))) < 1e-10 * abs(lhs)
    # finite differences in a few weight and bias entries
    b = RNG.standard_normal(4)
    f = lambda ww, bb: np.sum(nn.conv3x3(x, ww, bb) * dy)
    gw = nn.conv3x3_wgrad(x, dy)
    gb = nn.bias_grad(dy)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (3, 2, 1, 2), (1, 1, 2, 0)]:
        e = np.zeros_like(w)
        e[idx] = h
        fd = (f(w + e, b) - f(w - e, b)) / (2 * h)
        assert abs(fd - gw[idx]) < 1e-6 * max(1.0, abs(fd))
    e = np.zeros(4)
    e[2] = h
    assert abs((f(w, b + e) - f(w, b - e)) / (2 * h) - gb[2]) < 1e-6


def test_maxpool_and_upsample():
    x = RNG.standard_normal((2, 6, 4, 3))
    y = nn.maxpool2(x)
    for bi in range(2):
        for i in range(3):
            for j in range(2):
                for c in range(3):
                    assert y[bi, i, j, c] == x[bi, 2 * i:2 * i + 2, 2 * j:2 * j + 2, c].max()
    dy = RNG.standard_normal(y.shape)
    gx = nn.maxpool2_grad(x, dy)
    h = 1e-7  # no ties in random data: the max is differentiable
    for idx in [(0, 0, 0, 0), (1, 3, 2, 1), (0, 5, 3, 2), (1, 4, 1, 0)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (np.sum(nn.maxpool2(x + e) * dy) - np.sum(nn.maxpool2(x - e) * dy)) / (2 * h)
        assert abs(fd - gx[idx]) < 1e-6
    u = RNG.standard_normal((2, 3, 4, 5))
    v = RNG.standard_normal((2, 6, 8, 5))
    assert abs(np.sum(nn.upsample2(u) * v) - np.sum(u * nn.upsample2_grad(v))) < 1e-10
    assert np.array_equal(nn.upsample2(u)[:, 5, 7, :], u[:, 2, 3, :])


def test_nmse_loss_closed_forms_and_gradient():
    t = RNG.standard_normal((2, 4, 5, 6))
    loss, _ = nn.nmse_loss(np.zeros_like(t), t, 3)
    assert abs(loss - 1.0) < 1e-15           # o = 0: every band's ratio is 1
    loss, _ = nn.nmse_loss(2.0 * t, t, 3)
    assert abs(loss - 1.0) < 1e-15           # o = 2t likewise
    loss, g = nn.nmse_loss(t, t, 3)
    assert loss == 0.0 and np.all(g == 0.0)
    o = RNG.standard_normal(t.shape)
    loss, g = nn.nmse_loss(o, t, 3)
    h = 1e-7
    for idx in [(0, 0, 0, 0), (1, 3, 4, 5), (0, 2, 1, 3)]:
        e = np.zeros_like(o)
        e[idx] = h
        fd = (nn.nmse_loss(o + e, t, 3)[0] - nn.nmse_loss(o - e, t, 3)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-6


def test_nmse_loss_floor():
    """With a floor F_j in the denominators: o = 0 gives the mean of
    ||t_bj||^2 / (||t_bj||^2 + F_j); a zero floor is the plain loss; the
    gradient still matches finite differences."""
    t = RNG.standard_normal((2, 4, 5, 6))
    F = np.array([0.5, 3.0, 20.0])
    loss, _ = nn.nmse_loss(np.zeros_like(t), t, 3, floor=F)
    e = [np.sum(t[b, :, :, 2 * j:2 * j + 2] ** 2) for b in range(2) for j in range(3)]
    want = np.mean([e[3 * b + j] / (e[3 * b + j] + F[j]) for b in range(2) for j in range(3)])
    assert abs(loss - want) < 1e-15
    o = RNG.standard_normal(t.shape)
    assert nn.nmse_loss(o, t, 3, floor=np.zeros(3))[0] == nn.nmse_loss(o, t, 3)[0]
    loss, g = nn.nmse_loss(o, t, 3, floor=F)
    h = 1e-7
    for idx in [(0, 0, 0, 0), (1, 3, 4, 5)]:
        d = np.zeros_like(o)
        d[idx] = h
        fd = (nn.nmse_loss(o + d, t, 3, floor=F)[0] - nn.nmse_loss(o - d, t, 3, floor=F)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-6


def test_adam_closed_forms():
    # with a constant gradient the bias-corrected moments are g and g^2, so
    # every step moves each weight by lr g / (|g| + eps)
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 0.01
    for t in range(1, 6):
        w_new, m, v = nn.adam_step(w, g, m, v, t, lr)
        assert np.allclose(w - w_new, lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
        w = w_new


@pytest.fixture(scope="module")
def tiny():
    net = nn.UNetOracle(2, 3, (2, 3, 4, 5))
    p = {}
    for name, ci, co in net.layers:
        p[name] = (0.4 * RNG.standard_normal((co, 3, 3, ci)), 0.1 * RNG.standard_normal(co))
    x = RNG.standard_normal((2, 8, 8, 2))
    return net, p, x


def test_unet_shapes_and_skips(tiny):
    net, p, x = tiny
    y, c = net.forward(p, x)
    assert y.shape == (2, 8, 8, 3)
    assert c["d3a_in"].shape == (2, 2, 2, 9)    # upsampled w3 + skip w2
    assert c["d1a_in"].shape == (2, 8, 8, 5)    # upsampled w1 + skip w0


def test_unet_backward_by_finite_differences(tiny):
    net, p, x = tiny
    y, c = net.forward(p, x)
    dy = RNG.standard_normal(y.shape)
    g = net.backward(p, c, dy)
    h = 1e-6
    rng = np.random.default_rng(11)
    for name, ci, co in net.layers:
        w, b = p[name]
        for _ in range(2):
            idx = tuple(int(rng.integers(s)) for s in w.shape)
            e = np.zeros_like(w)
            e[idx] = h
            pp = dict(p)
            pp[name] = (w + e, b)
            fp = np.sum(net.forward(pp, x)[0] * dy)
            pp[name] = (w - e, b)
            fm = np.sum(net.forward(pp, x)[0] * dy)
            fd = (fp - fm) / (2 * h)
            assert abs(fd - g[name][0][idx]) < 1e-5 * max(1.0, abs(fd)), (name, idx)
        e = np.zeros_like(b)
        e[0] = h
        pp = dict(p)
        pp[name] = (w, b + e)
        fp = np.sum(net.forward(pp, x)[0] * dy)
        pp[name] = (w, b - e)
        fm = np.sum(net.forward(pp, x)[0] * dy)
        assert abs((fp - fm) / (2 * h) - g[name][1][0]) < 1e-5 * max(1.0, abs(fp - fm) / (2 * h)), name


def test_surrogate_maps_reconstruction_identity_and_zero_layer():
    """A last layer that hits its target exactly gives a decomposition that
    satisfies f = sum of bands + residual whenever the targets do (Eq. (7));
    a zero last layer gives bands 0, residual f and loss 1 per group; the
    input map sends [0, 1] to [-1, 1]."""
    B, H, W = 2, 5, 6
    f = RNG.random((B, 3, H, W))
    bands = 0.1 * RNG.standard_normal((B, 4, 3, H, W))
    res = f - bands.sum(axis=1)
    scale = np.linspace(0.5, 2.0, 15)
    t = nn.surrogate_target(f, bands, res)
    assert t.shape == (B, H, W, 15)
    out = nn.surrogate_output(t / scale, f, scale)
    assert np.allclose(out[:, :12].reshape(B, 4, 3, H, W), bands, atol=1e-15)
    assert np.allclose(out[:, 12:], res, atol=1e-15)
    assert np.allclose(out[:, :12].reshape(B, 4, 3, H, W).sum(axis=1) + out[:, 12:], f, atol=1e-14)
    z = nn.surrogate_output(np.zeros((B, H, W, 15)), f, scale)
    assert np.all(z[:, :12] == 0.0) and np.array_equal(z[:, 12:], f)
    loss, _ = nn.nmse_loss(np.zeros_like(t), t, 5)
    assert abs(loss - 1.0) < 1e-15
    assert np.all(nn.identity_error(f, out) < 1e-15) and np.all(nn.identity_error(f, z) == 0.0)
    # all-zero output: the error is the mean of |f|; a shift by d of one
    # band's channel adds |d| / 3
    e0 = nn.identity_error(f, np.zeros((B, 15, H, W)))
    assert np.allclose(e0, np.abs(f).mean(axis=(1, 2, 3)), rtol=0, atol=1e-15)
    sh = out.copy()
    sh[:, 4] += 0.3
    assert np.allclose(nn.identity_error(f, sh), 0.1, rtol=0, atol=1e-14)
    x = nn.surrogate_input(np.stack([np.zeros((3, H, W)), np.ones((3, H, W))]))
    assert x.shape == (2, H, W, 3) and np.all(x[0] == -1.0) and np.all(x[1] == 1.0)
