"""GPU tests of the C ABI's calling contract: the per-call report of
tvspec_decompose_ex, and calls on several streams at once.

Every result here is compared bit for bit with tvspec_decompose_dev's on the
same image and options (same kernels, same arithmetic); the decomposition
itself is checked against the oracle elsewhere, and once more here on the
report path.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2006_10004_amd import synth  # noqa: E402

CFG = dict(dt=0.005, K=24, iters=60, edges=[0, 1, 2, 4, 24])


@pytest.fixture(scope="module")
def tv():
    from paper_2006_10004_amd import tvspec
    assert torch.cuda.is_available()
    return tvspec


def to_np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def assert_same(a, b):
    for k in ("bands", "S", "residual"):
        assert np.array_equal(a[k], b[k]), k


def reference(tv, f, **kw):
    ft = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda()
    out = tv.tvspec_decompose_dev(ft, CFG["dt"], CFG["K"], CFG["iters"], CFG["edges"], **kw)
    torch.cuda.synchronize()
    return to_np(out)


def test_ex_device_report(tv, orc):
    f = synth.shapes_image(synth.ShapeSpec(96, 80, 1, 8), seed=5)
    ref = reference(tv, f)
    ft = torch.from_numpy(f).cuda()
    out, rep = tv.tvspec_decompose_ex(ft, CFG["dt"], CFG["K"], CFG["iters"], CFG["edges"])
    g = to_np(out)
    assert_same(g, ref)
    assert rep["recon_err"] == g["stats"][0] and rep["mean_err"] == g["stats"][1]
    assert rep["recon_err"] <= 1e-12 and rep["nonfinite"] == 0
    assert 0.0 < rep["device_ms"] <= rep["total_ms"]
    r = orc.decompose(f, CFG["dt"], CFG["K"], CFG["iters"], CFG["edges"])
    assert np.abs(g["bands"] - r["bands"]).max() <= 2e-4
    assert np.abs(g["residual"] - r["residual"]).max() <= 2e-4


@pytest.mark.parametrize("precision,ipl", [("mixed", 0), ("mixed", 4), ("mixed", 5), ("mixed", 8), ("mixed", 3),
                                           ("f64", 0), ("f32", 8)])
def test_ex_narrow_tiles_equal_square(tv, precision, ipl):
    """The 32 x 16 tile shape gives the 32 x 32 shape's results bit for bit
    (same per-pixel arithmetic), on a ragged 3-channel image: rows 70 = 4 x
    16 + 6, columns 45 = 32 + 13."""
    f = synth.shapes_image(synth.ShapeSpec(70, 45, 3, 6), seed=8)
    ref = reference(tv, f, precision=precision, iters_per_launch=ipl)
    ft = torch.from_numpy(f).cuda()
    out, _ = tv.tvspec_decompose_ex(ft, CFG["dt"], CFG["K"], CFG["iters"], CFG["edges"], precision=precision,
                                    iters_per_launch=ipl, tile_shape="narrow")
    assert_same(to_np(out), ref)


def test_ex_host_buffers_and_pdhg(tv):
    f = synth.shapes_image(synth.ShapeSpec(64, 72, 2, 6), seed=6)
    ref = reference(tv, f)
    out, rep = tv.tvspec_decompose_ex(f, CFG["dt"], CFG["K"], CFG["iters"], CFG["edges"])
    assert_same(out, ref)
    assert out["stats"][0] == rep["recon_err"] and rep["device_ms"] > 0.0
    # the primal-dual solver through the same entry equals its own entry point
    ft = torch.from_numpy(f).cuda()
    pd = tv.tvspec_decompose_pdhg_dev(ft, CFG["dt"], CFG["K"], CFG["iters"], CFG["edges"])
    torch.cuda.synchronize()
    out2, _ = tv.tvspec_decompose_ex(f, CFG["dt"], CFG["K"], CFG["iters"], CFG["edges"], solver="pdhg")
    assert_same(out2, to_np(pd))


def test_ex_nonfinite_device_input_with_report(tv):
    f = synth.shapes_image(synth.ShapeSpec(32, 32, 1, 3), seed=7)
    f[0, 3, 4] = np.inf
    ft = torch.from_numpy(f).cuda()
    with pytest.raises(tv.TvspecError) as ei:
        tv.tvspec_decompose_ex(ft, CFG["dt"], CFG["K"], CFG["iters"], CFG["edges"])
    assert ei.value.code == tv.TVSPEC_ENUMERIC
    # without a report the count is only in stats[2]
    out, rep = tv.tvspec_decompose_ex(ft, CFG["dt"], CFG["K"], CFG["iters"], CFG["edges"], report=False)
    torch.cuda.synchronize()
    assert rep is None and out["stats"][2].item() == 1.0


@pytest.mark.parametrize("precision", ["mixed", "f32"])
def test_calls_on_several_streams_at_once(tv, precision):
    """Three decompositions enqueued back to back without waiting, on two
    side streams and through the host entry's own stream, all sharing the
    library's scratch arena of one precision: each result equals the one
    computed alone."""
    imgs = [synth.shapes_image(synth.ShapeSpec(192, 160, 1, 12), seed=s) for s in (11, 12, 13)]
    alone = [reference(tv, f, precision=precision) for f in imgs]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    fts = [torch.from_numpy(f).cuda() for f in imgs]
    torch.cuda.synchronize()
    outs = []
    for f, st in ((fts[0], s1), (fts[1], s2)):
        with torch.cuda.stream(st):
            outs.append(tv.tvspec_decompose_dev(f, CFG["dt"], CFG["K"], CFG["iters"], CFG["edges"],
                                                precision=precision, stream=st))
    opts = dict(precision=precision)
    host_out, _ = tv.tvspec_decompose_ex(imgs[2], CFG["dt"], CFG["K"], CFG["iters"], CFG["edges"], **opts)
    torch.cuda.synchronize()
    assert_same(to_np(outs[0]), alone[0])
    assert_same(to_np(outs[1]), alone[1])
    assert_same(host_out, alone[2])
