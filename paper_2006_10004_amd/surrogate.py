"""The learned surrogate's pipeline around the library: training data from
the model-driven path, training, evaluation and serving with fallback.

Sec. 3 of the paper trains a network on decompositions the model-driven
method computes (its ground truth) and Sec. 4.3 compares their cost.  Here:

  make_images        seeded synthetic 3-channel shape images (synth.py)
  make_training_images  the training mix: serving-spec images and crops of
                     megapixel-spec images
  decompose_dataset  their decompositions by the batched GPU path
                     (tvspec_decompose_batch_dev) with the flow FLOW
  train              Adam steps of tvspec_net_train_step on random minibatches
  cosine_lr          the learning-rate schedule: linear warm-up, then cosine
                     decay to a floor
  band_errors        relative L1 error of predicted bands and residual
  SurrogateService   network inference with the reconstruction-identity check:
                     a result whose identity error exceeds the threshold is
                     replaced by the model-driven decomposition, and every
                     `judge_every`-th image is also decomposed by the
                     model-driven path to measure the surrogate's band error.

All arithmetic of the decomposition and of the network runs in the HIP
library; torch only holds device memory, gathers minibatches and computes
the evaluation metrics.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import synth, tvspec
from .nn import BANDS, IN_CHANNELS, OUT_CHANNELS, Net

# The decomposition the network learns: dt 0.005, K 100 samples, 150 inner
# iterations per ROF solve, 4 dyadic bands {0, 1, 2, 4, 100} and the residual.
FLOW = dict(dt=0.005, K=100, iters=150, edges=[0, 1, 2, 4, 100])

# Floor of the training loss's denominators (tvspec_net_set_loss_floor): 5%
# of the energy of a band at the dataset's RMS size.
LOSS_FLOOR = 0.05

# Gradient-norm clipping (tvspec_net_set_grad_clip): a step's gradient is
# scaled down to at most 2x the running average of gradient norms.  Floor
# 0.2 with clip 4 was measured too: held-out all-band relative L1 0.419,
# 0.439 and 0.479 over three minibatch orders, against 0.444, 0.445 and
# 0.457 here; the order alone moves the result by more than the setting.
GRAD_CLIP = 2.0

# Learning-rate schedule of the benchmark's training (cosine_lr): peak 3e-3
# after 500 warm-up steps, cosine decay to 1e-5.  Measured on the training
# mix (8192 images, batch 16, held-out all-band relative L1): constant 1e-3
# for 6000 steps 0.53; cosine from 1e-3, 6000 steps 0.53, 12000 steps 0.48;
# cosine from 2e-3, 12000 steps 0.48, 20000 steps 0.44; cosine from 3e-3,
# 12000 steps 0.46.  The error on training images is no lower than on
# held-out ones, so longer training helps and the network does not overfit.
LR_PEAK = 3e-3
LR_WARMUP = 500
LR_FLOOR = 1e-5


def cosine_lr(step, steps, peak=LR_PEAK, warmup=LR_WARMUP, floor=LR_FLOOR):
    """Learning rate of step `step` (0-based) of `steps`: linear warm-up to
    `peak` over `warmup` steps, then cosine decay to `floor` at the end."""
    if step < warmup:
        return peak * (step + 1) / warmup
    x = (step - warmup) / max(1, steps - warmup)
    return floor + 0.5 * (peak - floor) * (1.0 + np.cos(np.pi * min(1.0, x)))


def make_images(n, side, seed0, threads=16, spec=None):
    """n seeded images [n, 3, side, side] float32 (spec, by default
    synth.serving_spec(side))."""
    spec = spec or synth.serving_spec(side)
    out = np.empty((n, IN_CHANNELS, side, side), np.float32)

    def work(i):
        out[i] = synth.shapes_image(spec, seed0 + i)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, range(n)))
    return out


def make_training_images(n, side, seed0, threads=16, crop_from=4):
    """The surrogate's training mix, n images [n, 3, side, side] float32: the
    first half drawn with synth.serving_spec(side), the rest side x side
    crops (a crop_from x crop_from grid of tiles) of images drawn with
    synth.megapixel_spec(crop_from * side), so that the network also sees
    the local statistics of megapixel images (their noise level, dense
    and large shapes)."""
    n_a = (n + 1) // 2
    a = make_images(n_a, side, seed0, threads)
    per = crop_from * crop_from
    n_big = (n - n_a + per - 1) // per
    big = make_images(n_big, crop_from * side, seed0 + 1000003, threads,
                      spec=synth.megapixel_spec(crop_from * side))
    tiles = big.reshape(n_big, IN_CHANNELS, crop_from, side, crop_from, side).transpose(0, 2, 4, 1, 3, 5)
    tiles = tiles.reshape(n_big * per, IN_CHANNELS, side, side)[:n - n_a]
    return np.ascontiguousarray(np.concatenate([a, tiles]))


def decompose_dataset(f, flow=FLOW, chunk=64, precision="mixed"):
    """Bands [n, 4, 3, H, W] and residual [n, 3, H, W] (float64, on f's device)
    of the images f [n, 3, H, W] by the batched model-driven path."""
    n, C, H, W = f.shape
    bands = torch.empty((n, BANDS, C, H, W), dtype=torch.float64, device=f.device)
    res = torch.empty((n, C, H, W), dtype=torch.float64, device=f.device)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        outs = tvspec.tvspec_decompose_batch_dev(f[a:b].contiguous(), [flow["dt"]] * (b - a),
                                                 [flow["K"]] * (b - a), flow["iters"], [flow["edges"]] * (b - a),
                                                 precision=precision)
        for i, o in enumerate(outs):
            bands[a + i].copy_(o["bands"])
            res[a + i].copy_(o["residual"])
    return bands, res


def output_scales(bands, res):
    """Output scales [15]: the RMS of each band over a dataset (its three
    colour channels share it) and, for the residual's learned part (the
    residual minus f, i.e. minus the sum of the bands), the RMS of the sum of
    the bands."""
    s = np.empty(OUT_CHANNELS, np.float32)
    for j in range(BANDS):
        s[3 * j:3 * j + 3] = float(bands[:, j].pow(2).mean().sqrt())
    s[3 * BANDS:] = float(bands.sum(dim=1).pow(2).mean().sqrt())
    return s


def train(net, f, bands, res, steps, batch, lr, seed=0, loss_every=1):
    """`steps` Adam steps on minibatches drawn uniformly from the dataset;
    lr is a number or a function of the step index (0 .. steps - 1).
    Returns the losses of every loss_every-th step and of the last one; the
    steps in between are only enqueued, so the device runs ahead while the
    next minibatch is drawn."""
    g = torch.Generator().manual_seed(seed)
    n = f.shape[0]
    losses = []
    for i in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(f.device)
        rate = lr(i) if callable(lr) else lr
        sync = (i + 1) % loss_every == 0 or i == steps - 1
        loss = net.train_step(f.index_select(0, idx).contiguous(), bands.index_select(0, idx).contiguous(),
                              res.index_select(0, idx).contiguous(), float(rate), sync=sync)
        if sync:
            losses.append(loss)
    return losses


def split_output(out):
    """[B, 15, H, W] -> (bands [B, 4, 3, H, W], residual [B, 3, H, W])."""
    B, _, H, W = out.shape
    return out[:, :3 * BANDS].reshape(B, BANDS, IN_CHANNELS, H, W), out[:, 3 * BANDS:]


def band_errors(out, bands, res):
    """Relative L1 error sum|pred - ref| / sum|ref| per band and for the
    residual, over a batch; and the same over all bands together."""
    pb, pr = split_output(out)
    e = {}
    for j in range(BANDS):
        e["band%d" % (j + 1)] = float((pb[:, j].double() - bands[:, j]).abs().sum() / bands[:, j].abs().sum())
    e["residual"] = float((pr.double() - res).abs().sum() / res.abs().sum())
    e["all_bands"] = float((pb.double() - bands).abs().sum() / bands.abs().sum())
    return e


def conv_flops(H, W):
    """Multiply-add flops (2 per MAC) of one forward pass on an H x W image."""
    from .nn import LAYERS
    lvl = {"e1": 0, "e2": 1, "e3": 2, "e4": 3, "d3": 2, "d2": 1, "d1": 0, "ou": 0}
    total = 0
    for name, ci, co in LAYERS:
        s = 2 ** lvl[name[:2]]
        total += 2 * 9 * ci * co * (H // s) * (W // s)
    return total


class SurrogateService:
    """Decompositions by the network, with the model-driven path as fallback
    and as judge.

    - Identity check: an image whose reconstruction-identity error exceeds
      `threshold` (or is not finite) gets the model-driven decomposition.
    - Judge: every `judge_every`-th image (0 = never) is also decomposed by
      the model-driven path and the surrogate's band error measured against
      it (relative L1 over all bands; the surrogate's result is still the
      one served, so the judged error is the served error on a sample).
    - Consequence of the judge: per image size (H, W), the last `window`
      judged errors are kept; once at least `min_judged` of them average
      above `max_judged_l1`, that size is demoted and every later image of
      it is served by the model-driven path (reason "judged").  The identity
      error alone cannot see bands that are wrong but sum to the right
      image; the judge can.  `reset()` lifts every demotion (e.g. after the
      network is retrained)."""

    def __init__(self, net: Net, threshold=1e-2, judge_every=16, flow=FLOW, precision="mixed",
                 max_judged_l1=0.6, min_judged=4, window=32):
        self.net, self.threshold, self.judge_every = net, threshold, judge_every
        self.flow, self.precision = flow, precision
        self.max_judged_l1, self.min_judged, self.window = max_judged_l1, min_judged, window
        self.count = 0
        self.judged = []      # band-error dicts of judged images (with their size)
        self.fallbacks = 0    # images served by the model-driven path, any reason
        self.recent = {}      # (H, W) -> recent judged all-band errors
        self.demoted = set()  # sizes served by the model-driven path

    def reset(self):
        self.recent.clear()
        self.demoted.clear()

    def size_info(self):
        """Per image size: judged images in the window, their mean all-band
        error and whether the size is demoted."""
        return {"%dx%d" % k: {"judged": len(v), "mean_all_bands": float(np.mean(v)) if v else None,
                              "demoted": k in self.demoted} for k, v in self.recent.items()}

    def _plain(self, f):
        n = f.shape[0]
        fl = self.flow
        return tvspec.tvspec_decompose_batch_dev(f.contiguous(), [fl["dt"]] * n, [fl["K"]] * n, fl["iters"],
                                                 [fl["edges"]] * n, precision=self.precision)

    def _judge(self, size, err):
        w = self.recent.setdefault(size, [])
        w.append(err["all_bands"])
        del w[:-self.window]
        if len(w) >= self.min_judged and float(np.mean(w)) > self.max_judged_l1:
            self.demoted.add(size)

    def decompose(self, f):
        """f [B, 3, H, W] float32 -> dict(bands [B,4,3,H,W], residual [B,3,H,W]
        float32, source ['surrogate' | 'plain'] and reason [None |
        'identity' | 'judged'] per image, identity_error)."""
        B, _, H, W = f.shape
        size = (H, W)
        if size in self.demoted:
            plain = self._plain(f)
            self.count += B
            self.fallbacks += B
            bands = torch.stack([o["bands"] for o in plain]).float()
            res = torch.stack([o["residual"] for o in plain]).float()
            return {"bands": bands, "residual": res, "source": ["plain"] * B, "reason": ["judged"] * B,
                    "identity_error": np.full(B, np.nan)}
        out, err = self.net.forward(f, identity=True)
        err = err.cpu().numpy()
        bands, res = split_output(out)
        bands, res = bands.clone(), res.clone()
        src = ["surrogate"] * B
        reason = [None] * B
        fb = [i for i in range(B) if not (err[i] <= self.threshold)]
        jd = []
        if self.judge_every > 0:
            jd = [i for i in range(B) if (self.count + i) % self.judge_every == 0 and i not in fb]
        self.count += B
        todo = fb + jd
        if todo:
            idx = torch.tensor(todo, device=f.device)
            plain = self._plain(f.index_select(0, idx))
            for i, o in zip(todo, plain):
                if i in fb:
                    bands[i].copy_(o["bands"])
                    res[i].copy_(o["residual"])
                    src[i] = "plain"
                    reason[i] = "identity"
                else:
                    one = out[i:i + 1]
                    e = band_errors(one, o["bands"][None], o["residual"][None])
                    e["size"] = "%dx%d" % size
                    self.judged.append(e)
                    self._judge(size, e)
        self.fallbacks += len(fb)
        return {"bands": bands, "residual": res, "source": src, "reason": reason, "identity_error": err}


def timed(fn, *a, **k):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn(*a, **k)
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0
