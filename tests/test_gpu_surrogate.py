"""GPU tests of the surrogate's serving logic: the reconstruction-identity
check against the oracle's definition (Eq. (7)), the fallback to the
model-driven path when the check fails, and the sampled judging of the
surrogate's band error by that path.

The fallback results are compared with the batched model-driven path run on
each image alone: bit for bit, since its results do not depend on which
images share a launch.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import nn_oracle as orc_nn  # noqa: E402

DEV = "cuda:0"
FLOW = dict(dt=0.005, K=10, iters=20, edges=[0, 1, 2, 4, 10])


@pytest.fixture(scope="module")
def mods():
    from paper_2006_10004_amd import nn, surrogate, tvspec
    assert torch.cuda.is_available()
    return nn, surrogate, tvspec


def images(S, n, side, seed):
    return torch.from_numpy(S.make_images(n, side, seed)).to(DEV)


def plain_alone(tv, f):
    """Bands [4, 3, H, W] and residual [3, H, W] (float64) of each image by
    the batched model-driven path, one image per call."""
    out = []
    for i in range(f.shape[0]):
        o = tv.tvspec_decompose_batch_dev(f[i:i + 1].contiguous(), [FLOW["dt"]], [FLOW["K"]], FLOW["iters"],
                                          [FLOW["edges"]], precision="mixed")[0]
        out.append((o["bands"].clone(), o["residual"].clone()))
    return out


@pytest.mark.parametrize("B,H,W", [(1, 1, 1), (3, 17, 29), (2, 64, 64), (1, 256, 256)])
def test_identity_error_against_oracle(mods, B, H, W):
    nn = mods[0]
    rng = np.random.default_rng(B * H + W)
    f = rng.random((B, 3, H, W)).astype(np.float32)
    out = (0.05 * rng.standard_normal((B, 15, H, W))).astype(np.float32)
    out[:, 12:] += f
    err = nn.tvspec_net_identity_error(torch.from_numpy(f).to(DEV), torch.from_numpy(out).to(DEV)).cpu().numpy()
    ref = orc_nn.identity_error(f, out)
    assert np.allclose(err, ref, rtol=1e-5, atol=1e-7), (err, ref)


@pytest.mark.parametrize("H,W,B", [(8, 8, 1), (24, 40, 3), (256, 256, 2)])
def test_forward_checked_identity_error(mods, H, W, B):
    """The identity error computed while the output is written equals the
    oracle's on the stored output (up to the order of summation), and the
    output is the plain forward pass's, bit for bit."""
    nn = mods[0]
    net = nn.Net(H, W, 4, seed=7)
    p = net.get_params()
    net.set_params(p + 1e-3 * np.random.default_rng(8).standard_normal(p.size).astype(np.float32))
    net.set_output_scale(np.linspace(0.01, 0.1, 15).astype(np.float32))
    f = torch.from_numpy(np.random.default_rng(9).random((B, 3, H, W)).astype(np.float32)).to(DEV)
    out, err = net.forward(f, identity=True)
    plain = net.forward(f)
    assert torch.equal(out, plain)
    ref = orc_nn.identity_error(f.cpu().numpy(), out.cpu().numpy())
    assert np.allclose(err.cpu().numpy(), ref, rtol=1e-5, atol=0), (err, ref)
    alone = nn.tvspec_net_identity_error(f, out).cpu().numpy()
    assert np.allclose(err.cpu().numpy(), alone, rtol=1e-5, atol=0)
    net.close()


def perturbed(nn, scale, seed):
    net = nn.Net(64, 64, 4, seed=seed)
    p = net.get_params()
    net.set_params(p + scale * np.random.default_rng(seed).standard_normal(p.size).astype(np.float32))
    return net


def test_fresh_network_is_used_and_judged(mods):
    """Zero last layer: bands 0, residual f, identity error 0, so every image
    is served by the network; every second image is judged, and its band
    error against the model-driven path is exactly 1 (all bands zero)."""
    nn, S, tv = mods
    net = nn.Net(64, 64, 4, seed=1)
    f = images(S, 3, 64, 200)
    svc = S.SurrogateService(net, threshold=1e-2, judge_every=2, flow=FLOW)
    r = svc.decompose(f)
    assert r["source"] == ["surrogate"] * 3 and svc.fallbacks == 0
    assert np.all(r["identity_error"] == 0.0)
    assert torch.all(r["bands"] == 0) and torch.equal(r["residual"], f)
    assert len(svc.judged) == 2                      # images 0 and 2
    for e in svc.judged:
        assert e["all_bands"] == 1.0
    svc.decompose(images(S, 3, 64, 300))             # request count 3, 4, 5: 4 is judged
    assert len(svc.judged) == 3
    net.close()


def test_images_above_threshold_fall_back(mods):
    """With a threshold between the images' identity errors, those above it
    get the model-driven decomposition (the same as computed alone) and the
    others keep the network's output."""
    nn, S, tv = mods
    net = perturbed(nn, 2e-3, 5)
    f = images(S, 4, 64, 400)
    out = net.forward(f)
    err = nn.tvspec_net_identity_error(f, out).cpu().numpy()
    assert len(set(err.tolist())) == 4, err
    thr = float(np.sort(err)[1] + np.sort(err)[2]) / 2
    svc = S.SurrogateService(net, threshold=thr, judge_every=0, flow=FLOW)
    r = svc.decompose(f)
    fb = [i for i in range(4) if err[i] > thr]
    assert len(fb) == 2 and svc.fallbacks == 2 and not svc.judged
    alone = plain_alone(tv, f)
    for i in range(4):
        if i in fb:
            assert r["source"][i] == "plain"
            assert torch.equal(r["bands"][i], alone[i][0].float())
            assert torch.equal(r["residual"][i], alone[i][1].float())
        else:
            assert r["source"][i] == "surrogate"
            assert torch.equal(r["bands"][i].reshape(12, 64, 64), out[i, :12])
            assert torch.equal(r["residual"][i], out[i, 12:])
    net.close()


def test_non_finite_output_falls_back(mods):
    """A network whose output is NaN has a NaN identity error, which counts
    as a failed check."""
    nn, S, tv = mods
    net = nn.Net(64, 64, 4, seed=2)
    p = net.get_params()
    p[-1] = np.nan                                   # a bias of the last layer
    net.set_params(p)
    f = images(S, 2, 64, 500)
    svc = S.SurrogateService(net, threshold=1e-2, judge_every=0, flow=FLOW)
    r = svc.decompose(f)
    assert r["source"] == ["plain", "plain"]
    alone = plain_alone(tv, f)
    for i in range(2):
        assert torch.equal(r["bands"][i], alone[i][0].float())
    net.close()


def test_judged_error_demotes_the_size(mods):
    """The judged band error has a consequence: once the rolling mean of
    the judged errors of an image size exceeds the stated bound, later
    images of that size are served by the model-driven path (the same as
    computed alone), and reset() lifts it.  A fresh network (bands 0) is
    judged at error exactly 1."""
    nn, S, tv = mods
    net = nn.Net(64, 64, 4, seed=1)
    svc = S.SurrogateService(net, threshold=1e-2, judge_every=1, flow=FLOW, max_judged_l1=0.5, min_judged=2)
    r = svc.decompose(images(S, 2, 64, 600))
    assert r["source"] == ["surrogate"] * 2 and r["reason"] == [None, None]
    assert [e["all_bands"] for e in svc.judged] == [1.0, 1.0]
    assert svc.size_info()["64x64"] == {"judged": 2, "mean_all_bands": 1.0, "demoted": True}
    f = images(S, 3, 64, 700)
    r = svc.decompose(f)
    assert r["source"] == ["plain"] * 3 and r["reason"] == ["judged"] * 3
    alone = plain_alone(tv, f)
    for i in range(3):
        assert torch.equal(r["bands"][i], alone[i][0].float())
        assert torch.equal(r["residual"][i], alone[i][1].float())
    assert svc.fallbacks == 3
    svc.reset()
    r = svc.decompose(images(S, 1, 64, 800))
    assert r["source"] == ["surrogate"]
    net.close()


def test_judged_error_within_bound_keeps_the_network(mods):
    nn, S, tv = mods
    net = nn.Net(64, 64, 4, seed=1)
    svc = S.SurrogateService(net, threshold=1e-2, judge_every=1, flow=FLOW, max_judged_l1=1.5, min_judged=2)
    for seed in (900, 910, 920):
        r = svc.decompose(images(S, 2, 64, seed))
        assert r["source"] == ["surrogate"] * 2
    assert svc.size_info()["64x64"]["demoted"] is False and svc.fallbacks == 0
    net.close()
