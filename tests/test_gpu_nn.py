"""GPU parity of the surrogate network's kernels against the oracle
(oracle/nn_oracle.py).

Convolutions: inputs, weights and biases on the grid k/16, |k| <= 8, are
exact in bfloat16, their products are multiples of 1/256 and every sum here
stays below 2^24/256 in magnitude, so the float32 accumulation of the matrix
cores is exact: forward (float32 output), weight and bias gradients are
compared bit for bit with the float64 oracle, and the input gradient
(bfloat16 output) with the oracle rounded to bfloat16 (round to nearest
even, what the kernel's conversion does).

The whole network stores activations and their gradients in bfloat16
and its output in float32.  The oracle runs with the same storage
roundings (its act/out/grad hooks), so both sides take the same ReLU and
max-pooling decisions; what remains is float32 accumulation against float64
(relative ~1e-6 per sum), which moves a stored value across a bfloat16
rounding boundary only rarely, but then by one bfloat16 step (2^-8
relative), and the change propagates.  Output and loss are compared within
1e-2 relative L2.  A parameter gradient entry is a sum over all pixels of
terms of both signs that largely cancel (on the first layer its size is a
few per cent of the sum of the terms' sizes), so its error is judged
against that sum of sizes, sum_p |dz||x| (the oracle reports it): within
2e-2 in L2 norm, per layer.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import nn_oracle as orc_nn  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module")
def nn():
    from paper_2006_10004_amd import nn
    assert torch.cuda.is_available()
    return nn


def grid16(rng, shape):
    return rng.integers(-8, 9, size=shape).astype(np.float64) / 16.0


def bf(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).to(DEV)


def to_bf16_np(a):
    """float64 -> nearest bfloat16 (ties to even), back as float64."""
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("B,H,W,Cin,Cout,relu", [(2, 13, 19, 8, 16, False), (1, 9, 33, 48, 48, True),
                                                 (2, 16, 16, 144, 96, True), (1, 7, 5, 24, 64, False),
                                                 (2, 32, 40, 96, 192, True), (1, 24, 24, 576, 192, False),
                                                 # a partly filled channel block (NF 6, 80 channels) and a
                                                 # full one beside a partial one (112): the epilogue's
                                                 # element-by-element path
                                                 (1, 11, 37, 32, 80, True), (2, 9, 20, 16, 112, False),
                                                 # large grids
                                                 (2, 512, 512, 8, 96, True), (1, 512, 1024, 48, 48, False)])
def test_conv3x3_forward_exact(nn, B, H, W, Cin, Cout, relu):
    rng = np.random.default_rng(Cin * 7 + Cout)
    x = grid16(rng, (B, H, W, Cin))
    w = grid16(rng, (Cout, 3, 3, Cin))
    b = grid16(rng, (Cout,))
    ref = orc_nn.conv3x3(x, w, b)
    if relu:
        ref = orc_nn.relu(ref)
    y = nn.tvspec_nn_conv3x3(bf(x), bf(w), torch.from_numpy(b.astype(np.float32)).to(DEV), relu=relu,
                             out_f32=True)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy().astype(np.float64), ref)
    yb = nn.tvspec_nn_conv3x3(bf(x), bf(w), torch.from_numpy(b.astype(np.float32)).to(DEV), relu=relu)
    torch.cuda.synchronize()
    assert np.array_equal(yb.float().cpu().numpy().astype(np.float64), to_bf16_np(ref))


@pytest.mark.parametrize("B,H,W,Cout,Cin,masked", [(2, 13, 19, 16, 48, False), (1, 10, 12, 48, 144, True),
                                                   (2, 8, 8, 96, 16, True), (2, 24, 20, 192, 576, True),
                                                   # 80 input channels: a partly filled output block, the
                                                   # mask applied while staging
                                                   (2, 9, 20, 32, 80, True),
                                                   (2, 512, 512, 96, 16, True)])
def test_conv3x3_dgrad_exact(nn, B, H, W, Cout, Cin, masked):
    rng = np.random.default_rng(Cout * 5 + Cin)
    dy = grid16(rng, (B, H, W, Cout))
    w = grid16(rng, (Cout, 3, 3, Cin))
    ref = orc_nn.conv3x3_dgrad(dy, w)
    mask = None
    if masked:
        m = np.maximum(grid16(rng, (B, H, W, Cin)), 0.0)
        ref = ref * (m > 0)
        mask = bf(m)
    dx = nn.tvspec_nn_conv3x3_dgrad(bf(dy), bf(w), mask=mask)
    torch.cuda.synchronize()
    assert np.array_equal(dx.float().cpu().numpy().astype(np.float64), to_bf16_np(ref))


@pytest.mark.parametrize("B,H,W,Cin,Cout", [(2, 13, 19, 8, 16), (1, 9, 33, 48, 48), (2, 16, 16, 144, 96),
                                            (3, 24, 40, 16, 8),
                                            # 512 pixel ranges: the two-stage partial-sum reduction
                                            (2, 128, 128, 48, 48)])
def test_conv3x3_wgrad_exact(nn, B, H, W, Cin, Cout):
    rng = np.random.default_rng(Cin * 3 + Cout)
    x = grid16(rng, (B, H, W, Cin))
    dy = grid16(rng, (B, H, W, Cout))
    dw, db = nn.tvspec_nn_conv3x3_wgrad(bf(x), bf(dy))
    torch.cuda.synchronize()
    assert np.array_equal(dw.cpu().numpy().astype(np.float64), orc_nn.conv3x3_wgrad(x, dy))
    assert np.array_equal(db.cpu().numpy().astype(np.float64), orc_nn.bias_grad(dy))


def oracle_params(p, nn):
    """The parameters as the kernels use them: weights rounded to bfloat16
    from the float32 master copy, biases float32."""
    out = {}
    for name, (w, b) in nn.split_params(p).items():
        out[name] = (to_bf16_np(w.astype(np.float64)), b.astype(np.float64))
    return out


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def small_net(nn):
    net = nn.Net(32, 32, 2, seed=3)
    p = net.get_params()
    rng = np.random.default_rng(5)
    p = p + 0.02 * rng.standard_normal(p.size).astype(np.float32)  # non-zero biases too
    net.set_params(p)
    yield net, p
    net.close()


def inputs(seed, B=2, H=32, W=32):
    rng = np.random.default_rng(seed)
    f = rng.random((B, 3, H, W)).astype(np.float32)
    bands = 0.1 * rng.standard_normal((B, 4, 3, H, W))
    res = rng.random((B, 3, H, W))
    return f, bands, res


def test_params_round_trip(nn, small_net):
    net, p = small_net
    assert net.num_params == sum(co * 9 * ci + co for _, ci, co in nn.LAYERS)
    assert np.array_equal(net.get_params(), p)


def to_f32_np(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def stored_model():
    return orc_nn.UNetOracle(3, 15, (48, 96, 192, 384), act_store=to_bf16_np, out_store=to_f32_np,
                             grad_store=to_bf16_np)


def test_network_forward_against_oracle(nn, small_net):
    net, p = small_net
    f, _, _ = inputs(1)
    out = net.forward(torch.from_numpy(f).to(DEV))
    torch.cuda.synchronize()
    o = out.cpu().numpy().astype(np.float64)                          # [B,15,H,W]
    model = stored_model()
    # the network sees 2 f - 1 rounded to bfloat16
    x = to_bf16_np(orc_nn.surrogate_input(f))
    y, _ = model.forward(oracle_params(p, nn), x)
    ref = orc_nn.surrogate_output(y, f, np.ones(15))
    assert rel(o[:, :12], ref[:, :12]) < 1e-2, rel(o[:, :12], ref[:, :12])
    # the residual's learned part, without the f it adds
    assert rel(o[:, 12:] - f, ref[:, 12:] - f) < 1e-2


def test_network_forward_ragged_size_against_oracle(nn):
    """24 x 40 images: partial pixel tiles at every level (down to 3 x 5)
    and the decoder's in-place concatenation of odd-sized low levels."""
    net = nn.Net(24, 40, 2, seed=8)
    p = net.get_params()
    p = p + 0.02 * np.random.default_rng(6).standard_normal(p.size).astype(np.float32)
    net.set_params(p)
    f, _, _ = inputs(9, B=2, H=24, W=40)
    out = net.forward(torch.from_numpy(f).to(DEV))
    torch.cuda.synchronize()
    o = out.cpu().numpy().astype(np.float64)
    y, _ = stored_model().forward(oracle_params(p, nn), to_bf16_np(orc_nn.surrogate_input(f)))
    ref = orc_nn.surrogate_output(y, f, np.ones(15))
    assert rel(o[:, :12], ref[:, :12]) < 1e-2, rel(o[:, :12], ref[:, :12])
    assert rel(o[:, 12:] - f, ref[:, 12:] - f) < 1e-2
    net.close()


@pytest.mark.parametrize("side,B,sample", [(256, 16, (0, 11)), (512, 1, (0,))])
def test_network_forward_bench_configuration(nn, side, B, sample):
    """The inference configurations the benchmark times: batch 16 of
    3 x 256 x 256 shape images, and one 512 x 512 image (the large
    single-image grids of megapixel serving).  Sampled images of the batch
    are compared with the oracle, output and identity error."""
    from paper_2006_10004_amd import surrogate
    net = nn.Net(side, side, B, seed=13)
    p = net.get_params()
    p = p + 0.02 * np.random.default_rng(14).standard_normal(p.size).astype(np.float32)
    net.set_params(p)
    scale = np.linspace(0.005, 0.04, 15).astype(np.float32)
    net.set_output_scale(scale)
    f = surrogate.make_images(B, side, 300 + side)
    out, err = net.forward(torch.from_numpy(f).to(DEV), identity=True)
    torch.cuda.synchronize()
    o = out.cpu().numpy().astype(np.float64)
    e = err.cpu().numpy()
    model = stored_model()
    params = oracle_params(p, nn)
    for i in sample:
        fi = f[i:i + 1]
        y, _ = model.forward(params, to_bf16_np(orc_nn.surrogate_input(fi)))
        ref = orc_nn.surrogate_output(y, fi, scale)
        assert rel(o[i:i + 1, :12], ref[:, :12]) < 1e-2, (i, rel(o[i:i + 1, :12], ref[:, :12]))
        assert rel(o[i:i + 1, 12:] - fi, ref[:, 12:] - fi) < 1e-2
        ie = orc_nn.identity_error(fi, o[i:i + 1])[0]
        assert abs(e[i] - ie) <= 1e-5 * ie, (e[i], ie)
    net.close()


@pytest.mark.parametrize("side", [1024, 2048])
def test_network_forward_megapixel_crops(nn, side):
    """One megapixel image through a network of that size, as the megapixel
    service runs it (Net(side, side, 1)).  The network is translation
    equivariant away from the image border: crops whose offsets are
    multiples of 8 (so the pooling windows align) give the full image's
    output wherever the crop edge is more than the receptive field (~52 px)
    away.  So the interior [64, 192)^2 of a 256 x 256 crop, and [0, 192)^2 of
    the corner crop that shares the image border, are compared with the
    oracle network run on the crop."""
    from paper_2006_10004_amd import surrogate, synth
    net = nn.Net(side, side, 1, seed=17)
    p = net.get_params()
    p = p + 0.02 * np.random.default_rng(18).standard_normal(p.size).astype(np.float32)
    net.set_params(p)
    scale = np.linspace(0.005, 0.04, 15).astype(np.float32)
    net.set_output_scale(scale)
    f = surrogate.make_images(1, side, 900 + side, spec=synth.megapixel_spec(side))
    out = net.forward(torch.from_numpy(f).to(DEV))
    torch.cuda.synchronize()
    o = out.cpu().numpy().astype(np.float64)
    net.close()
    model = stored_model()
    params = oracle_params(p, nn)
    for y0, x0, lo in [(0, 0, 0), (side // 2 - 128, side // 2 + 64, 64)]:
        fc = np.ascontiguousarray(f[:, :, y0:y0 + 256, x0:x0 + 256])
        y, _ = model.forward(params, to_bf16_np(orc_nn.surrogate_input(fc)))
        ref = orc_nn.surrogate_output(y, fc, scale)[:, :, lo:192, lo:192]
        got = o[:, :, y0 + lo:y0 + 192, x0 + lo:x0 + 192]
        fr = fc[:, :, lo:192, lo:192]
        assert rel(got[:, :12], ref[:, :12]) < 1e-2, (y0, x0, rel(got[:, :12], ref[:, :12]))
        assert rel(got[:, 12:] - fr, ref[:, 12:] - fr) < 1e-2


@pytest.mark.parametrize("kappa", [0.0, 0.01])
def test_network_loss_and_gradients_against_oracle(nn, small_net, kappa):
    """kappa: the loss's denominator floor, kappa 3 H W scale_j^2 with the
    default output scales of 1."""
    net, p = small_net
    net.set_loss_floor(kappa)
    f, bands, res = inputs(2)
    loss, g = net.loss_grad(torch.from_numpy(f).to(DEV), torch.from_numpy(bands).to(DEV),
                            torch.from_numpy(res).to(DEV))
    model = stored_model()
    x = to_bf16_np(orc_nn.surrogate_input(f))
    params = oracle_params(p, nn)
    y, cache = model.forward(params, x)
    t = to_f32_np(orc_nn.surrogate_target(f, bands, res))
    ref_loss, dy = orc_nn.nmse_loss(y, t, 5, floor=np.full(5, kappa * 3 * 32 * 32))
    net.set_loss_floor(0.0)
    assert abs(loss - ref_loss) / ref_loss < 1e-2, (loss, ref_loss)
    scales = {}
    ref_g = model.backward(params, cache, to_bf16_np(dy), scales=scales)
    gs = nn.split_params(g)
    for name, _, _ in nn.LAYERS:
        for k in (0, 1):
            err = np.linalg.norm(gs[name][k] - ref_g[name][k]) / np.linalg.norm(scales[name][k])
            assert err < 2e-2, (name, k, err, rel(gs[name][k], ref_g[name][k]))


def test_training_reduces_the_loss(nn):
    """From the zero output layer (bands 0, residual f: loss 1 per group)
    the network learns targets that are a fixed linear function of the
    image."""
    net = nn.Net(32, 32, 2, seed=9)
    f, _, _ = inputs(3)
    c = (f - 0.5).astype(np.float64)
    bands = np.stack([0.1 * (j + 1) * c for j in range(4)], axis=1)
    res = f.astype(np.float64) - bands.sum(axis=1)
    ft, bt, rt = (torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (f, bands, res))
    first = net.train_step(ft, bt, rt, 1e-3)
    assert abs(first - 1.0) < 1e-6  # zero output layer
    for _ in range(100):
        last = net.train_step(ft, bt, rt, 1e-3)
    assert np.isfinite(last) and last < 0.5 * first, (first, last)
    net.close()


def test_output_scale_is_exact(nn):
    net = nn.Net(16, 16, 1, seed=6)
    p = net.get_params()
    net.set_params(p + 0.05 * np.random.default_rng(1).standard_normal(p.size).astype(np.float32))
    f = torch.from_numpy(inputs(7, B=1, H=16, W=16)[0]).to(DEV)
    a = net.forward(f).cpu().numpy()
    s = np.linspace(0.01, 2.0, 15).astype(np.float32)
    net.set_output_scale(s)
    b = net.forward(f).cpu().numpy()
    fn = f.cpu().numpy()
    # band channels: exactly scaled; residual: f + scale * (its learned part),
    # up to the float32 rounding of the additions of f
    assert np.array_equal(b[:, :12], a[:, :12] * s[None, :12, None, None])
    # a = fl(o + f), b = fl(fl(s o) + f) for the last layer's value o: b
    # differs from f + s (a - f) by at most 2^-24 (|b| + s |o| + s |a|)
    sr = s[None, 12:, None, None].astype(np.float64)
    ar, br = a[:, 12:].astype(np.float64), b[:, 12:].astype(np.float64)
    za = ar - fn
    bound = 2.0 ** -23 * (np.abs(br) + sr * np.abs(za) + sr * np.abs(ar))
    assert np.all(np.abs(br - (fn + za * sr)) <= bound)
    with pytest.raises(nn.TvspecError):
        net.set_output_scale(np.zeros(15, np.float32))
    net.close()


def test_adam_step_against_oracle(nn):
    """One training step moves every parameter by Adam's first step,
    lr * g / (|g| + eps) (float32 update of the float32 master weights)."""
    net = nn.Net(16, 16, 1, seed=4)
    p = net.get_params()
    net.set_params(p + 0.05 * np.random.default_rng(2).standard_normal(p.size).astype(np.float32))
    f, bands, res = inputs(4, B=1, H=16, W=16)
    ft, bt, rt = (torch.from_numpy(a).to(DEV) for a in (f, bands, res))
    p0 = net.get_params()
    _, g = net.loss_grad(ft, bt, rt)
    net.train_step(ft, bt, rt, 1e-3)
    p1 = net.get_params()
    w, _, _ = orc_nn.adam_step(p0.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, 1e-3)
    assert np.abs(p1 - w).max() < 1e-6
    net.close()


def test_training_is_deterministic(nn):
    """Every reduction (loss, weight and bias gradients, identity error) runs
    in a fixed order, so two networks from the same seed, trained on the same
    batches, end bit for bit equal; so do repeated forward passes."""
    f, bands, res = inputs(11, B=2, H=64, W=64)
    ft, bt, rt = (torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (f, bands, res))
    params, losses = [], []
    for _ in range(2):
        net = nn.Net(64, 64, 2, seed=21)
        net.set_output_scale(np.linspace(0.05, 0.5, 15).astype(np.float32))
        net.set_loss_floor(0.05)
        losses.append([net.train_step(ft, bt, rt, 1e-3) for _ in range(5)])
        params.append(net.get_params())
        a = net.forward(ft).cpu().numpy()
        b = net.forward(ft).cpu().numpy()
        assert np.array_equal(a, b)
        net.close()
    assert losses[0] == losses[1]
    assert np.array_equal(params[0], params[1])


def test_enqueued_training_steps_equal_synchronised_ones(nn):
    """Steps only enqueued (no loss read back) do the same work: the same
    parameters and, read afterwards with tvspec_net_last_loss, the same last
    loss as steps that each wait for their loss."""
    f, bands, res = inputs(12, B=2, H=64, W=64)
    ft, bt, rt = (torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (f, bands, res))
    params, last = [], []
    for sync in (True, False):
        net = nn.Net(64, 64, 2, seed=22)
        net.set_output_scale(np.linspace(0.05, 0.5, 15).astype(np.float32))
        net.set_grad_clip(2.0)
        out = [net.train_step(ft, bt, rt, 1e-3, sync=sync) for _ in range(6)]
        assert (out[-1] is not None) == sync
        last.append(net.last_loss())
        params.append(net.get_params())
        net.close()
    assert last[0] == last[1]
    assert np.array_equal(params[0], params[1])


def test_gradient_clipping(nn):
    """The first step's gradient norm is the norm of the gradient loss_grad
    returns and seeds the running average (no scaling); a batch whose
    gradient exceeds clip x average is scaled down to exactly that, and the
    average moves by 1% towards the clipped norm."""
    net = nn.Net(32, 32, 2, seed=17)
    p = net.get_params()
    net.set_params(p + 0.02 * np.random.default_rng(3).standard_normal(p.size).astype(np.float32))
    net.set_grad_clip(1.5)
    f, bands, res = inputs(12)
    ft, bt, rt = (torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (f, bands, res))
    _, g = net.loss_grad(ft, bt, rt)
    net.train_step(ft, bt, rt, 1e-3)
    norm, avg, scale = net.grad_stats()
    ref = np.linalg.norm(g.astype(np.float64))
    # the average is seeded with the norm, then updated as 0.99 n + 0.01 n
    # (float32 rounding)
    assert abs(norm - ref) / ref < 1e-6 and abs(avg - norm) < 1e-6 * norm and scale == 1.0
    # targets 30x smaller (bands and the residual's difference from f): the
    # normalised loss then has a much larger gradient
    net.train_step(ft, bt / 30.0, ft.double() + (rt - ft.double()) / 30.0, 1e-3)
    norm2, avg2, scale2 = net.grad_stats()
    lim = np.float32(1.5) * np.float32(avg)
    assert norm2 > lim
    assert abs(scale2 - lim / norm2) < 1e-6 * scale2
    assert abs(avg2 - (0.99 * avg + 0.01 * lim)) < 1e-6 * avg2
    with pytest.raises(nn.TvspecError):
        net.set_grad_clip(0.5)
    net.close()
