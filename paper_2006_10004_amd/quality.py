"""Quality of a decomposition against a reference one, with the measures the
paper evaluates its network by (its Appendix on evaluation measures; Table 1
reports their averages over the bands):

  PSNR    10 log10(MAX_I^2 / MSE(b, b_ref)); MAX_I is the largest intensity a
          band can take, 1 for images in [0, 1] (every band and the residual
          of such an image lie in [-1, 1]).
  SSIM    the structural similarity of Wang et al. (2004): luminance,
          contrast and structure terms from local means, variances and the
          covariance under an 11 x 11 Gaussian window of standard deviation
          1.5, with c1 = (0.01 L)^2, c2 = (0.03 L)^2, L = MAX_I, averaged
          over the window positions that fit inside the image (and over the
          colour channels).
  sLMSE   1 - LMSE(b, b_ref) / LMSE(0, b_ref), LMSE(b, b_ref) the sum over
          k x k patches at stride s of ||b_w - b_ref_w||^2 (k = 16, s = 8;
          patches start at multiples of s and must fit inside the image).

These are evaluation measures computed in float64 from the library's
outputs; they take no part in computing a decomposition.  Each function
takes est and ref of shape [N, C, H, W] (N images of one band, C colour
channels) and returns the N per-image values.
"""
from __future__ import annotations

import numpy as np
import torch

MAX_I = 1.0


def psnr(est: torch.Tensor, ref: torch.Tensor, max_i: float = MAX_I) -> np.ndarray:
    d = (est.double() - ref.double()).reshape(est.shape[0], -1)
    mse = d.pow(2).mean(dim=1).cpu().numpy()
    with np.errstate(divide="ignore"):
        return 10.0 * np.log10(max_i * max_i / mse)


def gaussian_window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    """Normalised 2-D Gaussian weights [size, size] (float64)."""
    x = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-(x * x) / (2.0 * sigma * sigma))
    g /= g.sum()
    return np.outer(g, g)


def ssim(est: torch.Tensor, ref: torch.Tensor, L: float = MAX_I, size: int = 11, sigma: float = 1.5) -> np.ndarray:
    x = est.double()
    y = ref.double()
    N, C, H, W = x.shape
    w = torch.from_numpy(gaussian_window(size, sigma)).to(x.device)[None, None]
    xs = x.reshape(N * C, 1, H, W)
    ys = y.reshape(N * C, 1, H, W)

    def blur(t):
        return torch.nn.functional.conv2d(t, w)

    mx, my = blur(xs), blur(ys)
    vx = blur(xs * xs) - mx * mx
    vy = blur(ys * ys) - my * my
    cxy = blur(xs * ys) - mx * my
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    m = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    return m.reshape(N, -1).mean(dim=1).cpu().numpy()


def lmse(est: torch.Tensor, ref: torch.Tensor, k: int = 16, s: int = 8) -> np.ndarray:
    """Sum over the k x k patches at stride s of the squared error, per image."""
    d = (est.double() - ref.double())
    N, C, H, W = d.shape
    if H < k or W < k:
        raise ValueError("images smaller than one %d x %d patch" % (k, k))
    sq = d.pow(2).sum(dim=1, keepdim=True)                       # [N, 1, H, W]
    ones = torch.ones((1, 1, k, k), dtype=sq.dtype, device=sq.device)
    return torch.nn.functional.conv2d(sq, ones, stride=s).reshape(N, -1).sum(dim=1).cpu().numpy()


def slmse(est: torch.Tensor, ref: torch.Tensor, k: int = 16, s: int = 8) -> np.ndarray:
    num = lmse(est, ref, k, s)
    den = lmse(torch.zeros_like(ref), ref, k, s)
    with np.errstate(divide="ignore", invalid="ignore"):
        return 1.0 - num / den


def band_quality(bands_est, bands_ref, res_est=None, res_ref=None):
    """The three measures per band (bands [N, B, C, H, W]) and for the
    residual ([N, C, H, W], optional), averaged over the N images, and their
    average over the bands ("bands_mean", as the paper's Table 1 reports)."""
    out = {}
    B = bands_ref.shape[1]
    for j in range(B):
        e, r = bands_est[:, j], bands_ref[:, j]
        out["band%d" % (j + 1)] = {"PSNR": float(np.mean(psnr(e, r))), "SSIM": float(np.mean(ssim(e, r))),
                                   "sLMSE": float(np.mean(slmse(e, r)))}
    if res_est is not None:
        out["residual"] = {"PSNR": float(np.mean(psnr(res_est, res_ref))),
                           "SSIM": float(np.mean(ssim(res_est, res_ref))),
                           "sLMSE": float(np.mean(slmse(res_est, res_ref)))}
    out["bands_mean"] = {m: float(np.mean([out["band%d" % (j + 1)][m] for j in range(B)]))
                         for m in ("PSNR", "SSIM", "sLMSE")}
    return out
