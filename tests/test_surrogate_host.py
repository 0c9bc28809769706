"""Host-side logic of the surrogate pipeline (paper_2006_10004_amd/surrogate.py):
the training-set mix, output scales, band errors and the flop count, checked
against their definitions on the CPU."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2006_10004_amd import surrogate as S, synth  # noqa: E402
from paper_2006_10004_amd.nn import LAYERS  # noqa: E402


def test_training_mix_is_serving_images_then_megapixel_crops():
    n, side = 21, 32
    mix = S.make_training_images(n, side, 40, threads=4)
    assert mix.shape == (n, 3, side, side) and mix.dtype == np.float32
    first = S.make_images(11, side, 40, threads=4)
    assert np.array_equal(mix[:11], first)
    big = S.make_images(1, 4 * side, 40 + 1000003, threads=4, spec=synth.megapixel_spec(4 * side))
    for i in range(n - 11):
        ty, tx = divmod(i, 4)
        assert np.array_equal(mix[11 + i], big[0, :, ty * side:(ty + 1) * side, tx * side:(tx + 1) * side])


def test_output_scales_are_band_rms():
    g = torch.Generator().manual_seed(0)
    bands = torch.randn((5, 4, 3, 8, 8), generator=g, dtype=torch.float64) * torch.tensor([1., 2., 3., 4.],
                                                                                           dtype=torch.float64
                                                                                           ).view(1, 4, 1, 1, 1)
    res = torch.randn((5, 3, 8, 8), generator=g, dtype=torch.float64)
    s = S.output_scales(bands, res)
    for j in range(4):
        want = math.sqrt(float((bands[:, j] ** 2).mean()))
        assert np.allclose(s[3 * j:3 * j + 3], want, rtol=1e-6)
    assert np.allclose(s[12:], math.sqrt(float((bands.sum(dim=1) ** 2).mean())), rtol=1e-6)


def test_band_errors_closed_forms():
    g = torch.Generator().manual_seed(1)
    bands = torch.randn((2, 4, 3, 6, 5), generator=g, dtype=torch.float64)
    res = torch.randn((2, 3, 6, 5), generator=g, dtype=torch.float64)
    exact = torch.cat([bands.reshape(2, 12, 6, 5), res], dim=1).float()
    e = S.band_errors(exact, bands, res)
    assert all(v < 1e-6 for v in e.values())
    e0 = S.band_errors(torch.zeros_like(exact), bands, res)
    assert all(abs(v - 1.0) < 1e-12 for v in e0.values())
    pb, pr = S.split_output(exact)
    assert pb.shape == (2, 4, 3, 6, 5) and pr.shape == (2, 3, 6, 5)


def test_conv_flops_of_the_encoder_decoder():
    total = 0
    for name, ci, co in LAYERS:
        lvl = {"e1": 0, "e2": 1, "e3": 2, "e4": 3, "d3": 2, "d2": 1, "d1": 0, "ou": 0}[name[:2]]
        total += 2 * 9 * ci * co * (256 >> lvl) ** 2
    assert S.conv_flops(256, 256) == total
    assert abs(total / 1e9 - 48.58) < 0.01


def test_cosine_lr_schedule():
    """Linear warm-up to the peak, then cosine decay that reaches the floor
    at the last step and never rises."""
    from paper_2006_10004_amd import surrogate as S
    steps, peak, warm, floor = 1000, 3e-3, 100, 1e-5
    lr = [S.cosine_lr(i, steps, peak, warm, floor) for i in range(steps + 1)]
    assert abs(lr[0] - peak / warm) < 1e-15 and abs(lr[warm - 1] - peak) < 1e-15
    assert all(abs(lr[i] - peak * (i + 1) / warm) < 1e-15 for i in range(warm))
    assert abs(lr[warm] - peak) < 1e-15
    assert abs(lr[steps] - floor) < 1e-15
    mid = warm + (steps - warm) // 2
    assert abs(lr[mid] - (floor + 0.5 * (peak - floor))) < 1e-12
    assert all(lr[i + 1] <= lr[i] + 1e-18 for i in range(warm, steps))
