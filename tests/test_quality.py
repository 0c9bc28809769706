"""Pins of the quality measures (paper_2006_10004_amd/quality.py) the
surrogate is evaluated by (the paper's Appendix on evaluation measures):
closed forms, and brute force by explicit window / patch loops on small
images (an implementation independent of the convolutions the module uses).
CPU only."""
import math

import numpy as np
import pytest
import torch

from paper_2006_10004_amd import quality as Q


def t(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float64))


def test_psnr_closed_forms():
    rng = np.random.default_rng(0)
    ref = rng.uniform(-1, 1, (3, 2, 17, 23))
    assert np.all(np.isinf(Q.psnr(t(ref), t(ref))))
    for c in (0.1, 0.01, 0.5):
        sign = np.where(rng.random(ref.shape) < 0.5, -1.0, 1.0)
        got = Q.psnr(t(ref + c * sign), t(ref))
        assert np.allclose(got, 20.0 * math.log10(1.0 / c), rtol=0, atol=1e-9)
    # a different peak scales the ratio: +20 dB for MAX_I x 10
    got = Q.psnr(t(ref + 0.1), t(ref), max_i=10.0)
    assert np.allclose(got, 40.0, atol=1e-9)


def test_gaussian_window():
    w = Q.gaussian_window(11, 1.5)
    assert w.shape == (11, 11) and abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1])
    # separable with weights proportional to exp(-x^2 / 4.5)
    assert abs(w[5, 6] / w[5, 5] - math.exp(-1.0 / 4.5)) < 1e-14


def ssim_brute(x, y, L=1.0, size=11, sigma=1.5):
    """Windowed SSIM by explicit loops over window positions and pixels."""
    w = Q.gaussian_window(size, sigma)
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    H, W = x.shape
    vals = []
    for i in range(H - size + 1):
        for j in range(W - size + 1):
            a = x[i:i + size, j:j + size]
            b = y[i:i + size, j:j + size]
            mx = float((w * a).sum())
            my = float((w * b).sum())
            vx = float((w * (a - mx) ** 2).sum())
            vy = float((w * (b - my) ** 2).sum())
            cxy = float((w * (a - mx) * (b - my)).sum())
            vals.append(((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2)))
    return float(np.mean(vals))


def test_ssim_against_brute_force():
    rng = np.random.default_rng(1)
    x = rng.uniform(-0.5, 0.5, (2, 3, 15, 19))
    y = x + 0.1 * rng.standard_normal(x.shape)
    got = Q.ssim(t(y), t(x))
    for n in range(2):
        ref = np.mean([ssim_brute(y[n, c], x[n, c]) for c in range(3)])
        assert abs(got[n] - ref) < 1e-12, (got[n], ref)


def test_ssim_closed_forms():
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (2, 1, 20, 20))
    assert np.allclose(Q.ssim(t(x), t(x)), 1.0, atol=1e-14)
    # constant images a and b: only the luminance term is left
    a, b = 0.3, -0.2
    c1 = 0.01 ** 2
    got = Q.ssim(t(np.full((1, 1, 12, 12), a)), t(np.full((1, 1, 12, 12), b)))
    assert abs(got[0] - (2 * a * b + c1) / (a * a + b * b + c1)) < 1e-12


def slmse_brute(est, ref, k=16, s=8):
    C, H, W = ref.shape
    num = den = 0.0
    for i in range(0, H - k + 1, s):
        for j in range(0, W - k + 1, s):
            num += float(((est[:, i:i + k, j:j + k] - ref[:, i:i + k, j:j + k]) ** 2).sum())
            den += float((ref[:, i:i + k, j:j + k] ** 2).sum())
    return 1.0 - num / den


def test_slmse_against_brute_force():
    rng = np.random.default_rng(3)
    ref = rng.standard_normal((2, 3, 41, 33))
    est = ref + 0.3 * rng.standard_normal(ref.shape)
    got = Q.slmse(t(est), t(ref))
    for n in range(2):
        assert abs(got[n] - slmse_brute(est[n], ref[n])) < 1e-12


def test_slmse_closed_forms():
    rng = np.random.default_rng(4)
    ref = rng.standard_normal((3, 2, 32, 48))
    assert np.allclose(Q.slmse(t(ref), t(ref)), 1.0)
    assert np.allclose(Q.slmse(t(np.zeros_like(ref)), t(ref)), 0.0)
    assert np.allclose(Q.slmse(t(2 * ref), t(ref)), 0.0)
    for a in (0.1, 0.5, 0.9):   # LMSE scales with the square of the error
        assert np.allclose(Q.slmse(t((1 - a) * ref), t(ref)), 1 - a * a, atol=1e-12)
    # one patch position per axis when the image is exactly one patch wide
    one = rng.standard_normal((1, 1, 16, 16))
    e = one + 0.2
    assert abs(Q.slmse(t(e), t(one))[0] - (1 - 0.04 * 256 / float((one ** 2).sum()))) < 1e-12
    with pytest.raises(ValueError):
        Q.lmse(t(np.zeros((1, 1, 15, 40))), t(np.zeros((1, 1, 15, 40))))


def test_band_quality_averages():
    rng = np.random.default_rng(5)
    ref = rng.uniform(-0.2, 0.2, (2, 4, 3, 32, 32))
    est = ref.copy()
    est[:, 1] += 0.01
    q = Q.band_quality(t(est), t(ref), t(ref[:, 0]), t(ref[:, 0]))
    assert math.isinf(q["band1"]["PSNR"]) and q["band1"]["SSIM"] == pytest.approx(1.0)
    assert q["band2"]["PSNR"] == pytest.approx(40.0)
    assert q["bands_mean"]["sLMSE"] == pytest.approx(np.mean([q["band%d" % j]["sLMSE"] for j in (1, 2, 3, 4)]))
    assert q["residual"]["sLMSE"] == pytest.approx(1.0)
