"""The allocation-free entry point (tvspec_decompose_noalloc_dev) against
tvspec_decompose_dev: same kernels and arithmetic, so the results must be
equal bit for bit, on consecutive calls that reuse the library's fixed
scratch array with a smaller image the second time."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2006_10004_amd import synth  # noqa: E402


@pytest.fixture(scope="module")
def tv():
    from paper_2006_10004_amd import tvspec
    assert torch.cuda.is_available()
    return tvspec


def outputs(K, C, H, W, nb):
    z = lambda *s: torch.full(s, float("nan"), dtype=torch.float64, device="cuda:0")
    return {"bands": z(nb, C, H, W), "S": z(C, K), "residual": z(C, H, W), "stats": z(4)}


def both(tv, f, dt, K, iters, edges, **kw):
    ft = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    C, H, W = ft.shape
    print("noalloc case: C=%d H=%d W=%d K=%d iters=%d %s" % (C, H, W, K, iters, kw), flush=True)
    ref = tv.tvspec_decompose_dev(ft, dt, K, iters, edges, **kw)
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy() for k, v in ref.items()}
    out = tv.tvspec_decompose_noalloc_dev(ft, dt, K, iters, edges, outputs(K, C, H, W, len(edges) - 1), **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, ref


def assert_equal(g, r):
    for k in ("bands", "S", "residual", "stats"):
        assert np.array_equal(g[k], r[k]), k


@pytest.mark.parametrize("precision", ["mixed", "f32", "f64"])
def test_noalloc_two_calls_second_smaller(tv, precision):
    big = synth.shapes_image(synth.ShapeSpec(176, 144, 2, 14), seed=21)
    small = synth.shapes_image(synth.ShapeSpec(70, 90, 1, 6), seed=22)
    g, r = both(tv, big, 0.005, 24, 60, [0, 1, 2, 4, 8, 24], precision=precision)
    assert_equal(g, r)
    assert g["stats"][0] <= 1e-12 and g["stats"][2] == 0
    g, r = both(tv, small, 0.004, 12, 45, [0, 1, 12], precision=precision)
    assert_equal(g, r)
    assert g["stats"][0] <= 1e-12 and g["stats"][2] == 0


def test_noalloc_counter_cleared_between_calls(tv):
    """A call on an image with one infinity counts it; the next call on a
    clean image reports zero (the counter in the shared array is cleared)."""
    bad = synth.shapes_image(synth.ShapeSpec(40, 48, 1, 4), seed=23)
    bad[0, 5, 7] = np.inf
    ft = torch.from_numpy(bad).cuda()
    out = tv.tvspec_decompose_noalloc_dev(ft, 0.005, 6, 20, [0, 6], outputs(6, 1, 40, 48, 1))
    torch.cuda.synchronize()
    assert out["stats"][2].item() == 1.0
    clean = synth.shapes_image(synth.ShapeSpec(32, 40, 1, 4), seed=24)
    g, r = both(tv, clean, 0.005, 6, 20, [0, 1, 6])
    assert_equal(g, r)
    assert g["stats"][2] == 0


def test_noalloc_full_512_workload_equals_dev(tv):
    """The benchmark's 512x512 single-plane workload shape fits the array:
    a shortened flow (K = 16) at the full size, in the launch configuration
    the benchmark times (automatic blocking)."""
    f = synth.shapes_image(synth.IMAGE_512, seed=0)
    g, r = both(tv, f, 0.002, 16, 300, [0, 1, 2, 4, 8, 16])
    assert_equal(g, r)


def test_noalloc_rejects_oversize(tv):
    f = torch.zeros((1, 2048, 2048), dtype=torch.float32, device="cuda:0")
    out = outputs(4, 1, 2048, 2048, 1)
    with pytest.raises(tv.TvspecError) as ei:
        tv.tvspec_decompose_noalloc_dev(f, 0.01, 4, 10, [0, 4], out)
    assert ei.value.code == tv.TVSPEC_EINVAL and "bytes of scratch" in str(ei.value)
