#!/usr/bin/env python3
"""Benchmark of the plain spectral-TV decomposition on one MI355X.

    python bench.py [--steps K] [--warmup W] [--precision f32|f64]

One step = one whole decomposition (K+1 ROF solves by Chambolle iterations,
phi, S, bands, residual and the reconstruction check) of the 512 x 512
greyscale synthetic shape image (40 disks / rectangles / ellipses, radius
U[3,120], contrast U[-0.6,0.6], noise sigma 0.03), dt = 0.002, K = 200
spectral samples, 300 Chambolle iterations per solve, tau = 0.248, 8 dyadic
bands.  The image is resident in HBM before the timed region starts.

Prints ONE JSON line: throughput (MPix/s), p50/p99 latency, the roofline of
the dominant kernel (the Chambolle iteration kernel, timed live with hipEvents
around every launch in a separate pass over the same workload) and the FP64
CPU oracle timed on this host's cores.
"""
import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = {
    "workload": "512x512 greyscale synthetic shapes (40 disks/rects/ellipses), plain TV-flow "
                "spectral decomposition",
    "H": 512, "W": 512, "C": 1, "seed": 0,
    "dt": 0.002, "K": 200, "inner_iters": 300, "n_bands": 8, "tau": 0.248,
}
# algorithmic HBM bytes of one Chambolle pixel-iteration: read the dual field
# (px, py) and the data term G = grad(g)/dt (Gx, Gy), write (px, py); the
# dual field is float32 in F32 and float64 in MIXED and F64, G is float32 in
# F32 and MIXED and float64 in F64
BYTES_PER_PIXEL_ITER = {"f32": 24, "mixed": 40, "f64": 48}
# the same for the primal-dual kernel: read x, xbar, y (2) and the data u_k
# (float64), write x, xbar, y (2); the iterates are float32 in F32, float64
# otherwise
PDHG_BYTES_PER_PIXEL_ITER = {"f32": 40, "mixed": 72, "f64": 72}
# algorithmic floating-point operations of one Chambolle pixel-iteration, as
# the method states the update (square root and division counted as one
# operation each): div p (3), w = div p - g/dt (1, g/dt formed once per
# solve), grad w (2), |grad w| (2 mul, 1 add, 1 sqrt), 1 + tau |grad w| (2),
# p + tau grad w (4), the division of both components (2)
FLOPS_PER_PIXEL_ITER = 18
# the same for a primal-dual pixel-iteration: grad xbar (2), y + sigma grad
# xbar (4), |z| (4), min(1, dt/|z|) (2), scaling (2), div y (3), x + tau div y
# + tau g (4), / (1 + tau) (1), xbar = 2x' - x (2)
PDHG_FLOPS_PER_PIXEL_ITER = 24
# vector peaks (MI355X, 256 CUs at 2.4 GHz): FP64 78.6 TFLOP/s, FP32 157.3
ALU_PEAK_TFLOPS = {"f32": 157.3, "mixed": 78.6, "f64": 78.6}
# arithmetic type of the path, per precision mode
DTYPE = {"f32": "f32", "mixed": "f64 (f32-seeded sqrt/rcp)", "f64": "f64"}
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# The band error the surrogate is served at: a size whose rolling judged
# all-band relative L1 error exceeds it goes to the plain path.
SURROGATE_MAX_JUDGED_L1 = 0.6


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_chambolle_tile_512x512_mixed_traffic.md")
PDHG_TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_pdhg_tile_512x512_mixed_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2006_10004_amd", "csrc", "tile_kernels.h")


def measured_traffic(precision, iters_per_launch, record=TRAFFIC_RECORD):
    """HBM bytes per tile-kernel launch from a committed counter record (the
    Chambolle tile's by default), or None when the record is for another
    configuration or the kernel source has changed since the counters were
    taken."""
    import hashlib
    import re
    if precision != "mixed" or iters_per_launch not in (0, 8) or not os.path.exists(record):
        return None
    m = re.search(r"```json\s*(\{.*?\})\s*```", open(record).read(), flags=re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None
    return rec["traffic_bytes_per_launch"]


def alu_roofline(kernel, t, ms_per_step, precision, flops_per_pit, bytes_per_pit, traffic):
    """Roofline record of a temporally blocked tile kernel from its live
    timing t (summed kernel ms, launches, pixel-iterations).  The kernel
    keeps its region on chip for several iterations, so HBM does not bound
    it (the counters' traffic is a fraction of one unblocked pass); what
    does is vector-ALU issue.  achieved = algorithmic floating-point
    operations per launch / average launch duration, against the vector
    peak of the mode's arithmetic type.  Beside it: the measured HBM rate
    (counter bytes per launch / duration) and the effective rate of an
    unblocked kernel moving bytes_per_pit per pixel-iteration."""
    avg_s = t["kernel_ms"] / t["launches"] / 1e3
    pit = t["pixel_iters"] / t["launches"]
    achieved = flops_per_pit * pit / avg_s / 1e12
    peak = ALU_PEAK_TFLOPS[precision]
    rec = {
        "kernel": kernel,
        "bound": "alu",
        "achieved": achieved,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": traffic,
        "flops_per_pixel_iter": flops_per_pit,
        "pixel_iters_per_launch": pit,
        "avg_launch_us": avg_s * 1e6,
        "launches_per_step": t["launches"],
        "kernel_share_of_step": t["kernel_ms"] / ms_per_step,
        "hbm_GBps": traffic / avg_s / 1e9 if traffic else None,
        "hbm_frac": traffic / avg_s / 1e9 / HBM_PEAK_GBS if traffic else None,
        "effective_GBps": bytes_per_pit * pit / avg_s / 1e9,
    }
    return rec


def whole_job_alu(pixel_iters, seconds, precision="mixed"):
    """The whole-job counterpart of the kernel roofline: 18 flops per
    pixel-iteration (one Chambolle update) over the job's wall time, against
    the vector-ALU peak of the mode.  It includes every idle gap, queueing
    and the per-solve kernels, so it bounds the tile kernel's own fraction
    from below."""
    tf = FLOPS_PER_PIXEL_ITER * pixel_iters / seconds / 1e12
    return {"pixel_iters": pixel_iters, "achieved_TFLOPs": tf, "peak_TFLOPs": ALU_PEAK_TFLOPS[precision],
            "frac": tf / ALU_PEAK_TFLOPS[precision], "kind": "whole job (wall time)"}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_model():
    """The host CPU as /proc/cpuinfo names it: model name, vendor, family,
    model and stepping, and the logical CPUs this process may use (a virtual
    machine may report only a generic model name, so the numbers are kept
    beside it)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = line.split(":", 1)
                info.setdefault(k.strip(), v.strip())
    except OSError:
        return None
    name = info.get("model name")
    if not name:
        return None
    parts = [name]
    ids = ["%s %s" % (k, info[k]) for k in ("vendor_id", "cpu family", "model", "stepping") if k in info]
    if ids:
        parts.append("(" + ", ".join(ids) + ")")
    try:
        parts.append("%d logical CPUs available" % len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        pass
    return " ".join(parts)


def cpu_baseline(f, wl, one_thread_steps=12, others=True):
    """Time the FP64 CPU oracle on the full workload (all host threads), and
    on one thread over the first `one_thread_steps` flow steps of the same
    workload (a child process with OMP_NUM_THREADS=1), scaled per ROF solve
    to the full workload."""
    import subprocess
    import tempfile
    import numpy as np
    import oracle
    edges = oracle.dyadic_edges(wl["K"], wl["n_bands"])
    t0 = time.perf_counter()
    oracle.decompose(f, wl["dt"], wl["K"], wl["inner_iters"], edges, tau=wl["tau"])
    sec = time.perf_counter() - t0
    mpix = wl["H"] * wl["W"] * wl["C"] / 1e6
    rec = {"value": mpix / sec, "unit": "MPix/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": "one full decomposition of the same %dx%d workload (%d ROF solves x %d "
                     "iterations), %.1f s" % (wl["H"], wl["W"], wl["K"] + 1, wl["inner_iters"], sec),
           "cpu_model": cpu_model()}
    k1 = one_thread_steps
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "f.npy")
        np.save(path, f)
        code = ("import sys, time, numpy as np; sys.path.insert(0, %r); import oracle; f = np.load(%r); "
                "t0 = time.perf_counter(); oracle.decompose(f, %r, %d, %d, [0, %d], tau=%r); "
                "print(time.perf_counter() - t0)" % (ROOT, path, wl["dt"], k1, wl["inner_iters"], k1, wl["tau"]))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        print("one-thread oracle sample failed:\n" + r.stderr[-2000:], file=sys.stderr)
    else:
        s1 = float(r.stdout.strip().splitlines()[-1])
        full1 = s1 * (wl["K"] + 1) / (k1 + 1)
        rec["one_thread"] = {"value": mpix / full1, "unit": "MPix/s", "cores": 1,
                             "sample": "the first %d flow steps (%d ROF solves x %d iterations), %.1f s, scaled per "
                                       "solve to the %d solves of the workload" % (k1, k1 + 1, wl["inner_iters"], s1,
                                                                                   wl["K"] + 1)}
    if others:
        rec["other_workloads"] = oracle_other_workloads()
    return rec


def oracle_other_workloads(mega_steps=2):
    """The oracle (all host threads) on the two other plain-path workloads:
    the 64x64 parity workload in full, and the 3x1024x1024 megapixel flow
    (dt 0.002, K 300, 200 iterations) over its first `mega_steps` flow
    steps, scaled per ROF solve to the 301 solves of the full call."""
    import oracle
    from paper_2006_10004_amd import synth
    out = {}
    f64 = synth.shapes_image(synth.SMALL_64, 0)
    t0 = time.perf_counter()
    oracle.decompose(f64, 0.005, 60, 200, [0, 1, 2, 4, 60], tau=WORKLOAD["tau"])
    s = time.perf_counter() - t0
    out["64x64"] = {"value": 64 * 64 / 1e6 / s, "unit": "MPix/s", "cores": oracle.num_threads(), "seconds": s,
                    "sample": "one full decomposition of the 64x64 workload (dt 0.005, K 60, 61 ROF solves x 200 "
                              "iterations)"}
    fm = synth.shapes_image(synth.megapixel_spec(1024), 61000)
    t0 = time.perf_counter()
    oracle.decompose(fm, 0.002, mega_steps, 200, [0, mega_steps], tau=WORKLOAD["tau"])
    s = time.perf_counter() - t0
    full = s * 301 / (mega_steps + 1)
    out["3x1024x1024"] = {"value": 1024 * 1024 / 1e6 / full, "unit": "MPix/s", "cores": oracle.num_threads(),
                          "seconds_full_estimate": full,
                          "sample": "the first %d flow steps of the megapixel flow (dt 0.002, %d ROF solves x 200 "
                                    "iterations on 3 x 1024 x 1024), %.1f s, scaled per solve to the 301 solves of "
                                    "K = 300" % (mega_steps, mega_steps + 1, s)}
    return out


def pdhg_block(f, wl, edges, precision, steps):
    """The same workload with the primal-dual inner solver (steps
    1/sqrt(8)): time per decomposition, throughput and the roofline of its
    tile kernel."""
    import torch
    from paper_2006_10004_amd import tvspec

    def run(out=None):
        return tvspec.tvspec_decompose_pdhg_dev(f, wl["dt"], wl["K"], wl["inner_iters"], edges,
                                                precision=precision, out=out)

    out = run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run(out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    tvspec.tvspec_timing_enable(True)
    try:
        run(out)
        torch.cuda.synchronize()
        t = tvspec.tvspec_timing_read()
    finally:
        tvspec.tvspec_timing_enable(False)
    st = out["stats"].cpu().numpy()
    px = wl["H"] * wl["W"] * wl["C"]
    return {"solver": "pdhg (Chambolle-Pock, tau = sigma = 1/sqrt(8))", "ms_per_step": ms,
            "MPix_per_s": px / 1e6 / (ms / 1e3), "steps": steps,
            "roofline": alu_roofline("k_pdhg_tile", t, ms, precision, PDHG_FLOPS_PER_PIXEL_ITER,
                                     PDHG_BYTES_PER_PIXEL_ITER[precision],
                                     measured_traffic(precision, 0, PDHG_TRAFFIC_RECORD)),
            "report": {"recon_err": float(st[0]), "mean_err": float(st[1])}}


def other_precisions(f, wl, edges, ref, steps=2):
    """The same workload in the other two precision modes of the inner
    iteration: time per decomposition (one untimed call, then `steps` back
    to back) and the distance of the bands and S from the reference output
    (the headline mode's; its own distance from the float64 oracle is
    asserted by the GPU tests)."""
    import torch
    from paper_2006_10004_amd import tvspec
    res = {}
    for prec in ("f32", "mixed", "f64"):
        if prec == wl["precision"]:
            continue

        def run(out=None):
            return tvspec.tvspec_decompose_dev(f, wl["dt"], wl["K"], wl["inner_iters"], edges, out=out,
                                               tau=wl["tau"], precision=prec)

        out = run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run(out)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        px = wl["H"] * wl["W"] * wl["C"]
        res[prec] = {"ms_per_step": ms, "MPix_per_s": px / 1e6 / (ms / 1e3), "dtype": DTYPE[prec],
                     "bands_max_abs_vs_headline": float((out["bands"] - ref["bands"]).abs().max()),
                     "S_rel_peak_vs_headline": float((out["S"] - ref["S"]).abs().max() / ref["S"].abs().max())}
    return res


def batch_throughput(n, precision):
    """One batched call over n seeded 64x64 shape images (dt 0.005, K 60, 200
    iterations, 4 dyadic bands): MPix/s of the whole batch."""
    import numpy as np
    import torch
    from paper_2006_10004_amd import synth, tvspec
    imgs = np.stack([synth.shapes_image(synth.SMALL_64, 1000 + i) for i in range(n)])
    f = torch.from_numpy(imgs).to("cuda:0")
    edges = [[0, 1, 2, 4, 60]] * n

    def call():
        return tvspec.tvspec_decompose_batch_dev(f, [0.005] * n, [60] * n, 200, edges, precision=precision)

    call()
    torch.cuda.synchronize()
    # Python's cyclic collector is paused over the timed calls (as timeit
    # does): each call builds a few thousand small objects (one dict of
    # tensor views per image), and a full collection landing inside a call
    # stalls the submission of the next for ~30 ms, which is the
    # interpreter's time, not the library's.
    gc_was_on = gc.isenabled()
    gc.collect()
    gc.disable()
    try:
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
    finally:
        if gc_was_on:
            gc.enable()
    return {"images": n, "ms_per_batch": ms, "MPix_per_s": n * 64 * 64 / 1e6 / (ms / 1e3),
            "workload": "64x64 shape images, dt 0.005, K 60, 200 iterations, 4 dyadic bands"}


SERVING = {
    "workload": "continuous-batching server, 3-channel synthetic shape images (40 shapes, size scaled "
                "with the side), side uniform in {128, 256, 512, 1024}, Poisson arrivals",
    "C": 3, "sides": [128, 256, 512, 1024], "dt": 0.005, "K": 100, "inner_iters": 150, "n_bands": 4,
}
# A second Poisson run at a fixed arrival rate, so that latency percentiles
# compare across builds at one offered load (the other run's rate follows
# the measured burst throughput).  12.6 requests/s is 85% of the burst
# throughput of the server that replayed one solve per graph (14.8/s).
SERVING_FIXED_RATE = 12.6
SERVING_FIXED_REQUESTS = 384


MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16

# The paper's own timing (Table 3; NVIDIA Quadro P6000, 1024 x 1024 images,
# seconds per image): the model-driven primal-dual GPU implementation against
# its networks.  Context for the surrogate's speedup only: other hardware,
# other flow parameters, a plain path ~40x slower than this one.
PAPER_1024_CONTEXT = {"hardware": "NVIDIA Quadro P6000", "pixels": 1048576, "model_driven_gpu_s": 28.2811,
                      "tvspecnet_s": 0.0020, "u_tvspecnet_s": 0.0062,
                      "speedup_tvspecnet": 28.2811 / 0.0020, "speedup_u_tvspecnet": 28.2811 / 0.0062}


def surrogate_block(n_train, steps, test_images=64, batch=16, lr=3e-3, mega_sides=(1024, 2048), mega_requests=8,
                    seed=11):
    """The learned surrogate end to end on the surrogate workload: training
    data decomposed by the batched plain path (3 x 256^2 shape images,
    dt 0.005, K 100, 150 iterations, 4 dyadic bands), `steps` Adam steps
    (batch 16, learning rate: 500 warm-up steps to `lr`, then cosine decay to
    1e-5), band errors on held-out images, inference
    throughput against the bf16 MFMA peak, serving with identity-error
    fallback; then megapixel serving: `mega_requests` images alternating
    over mega_sides (300 shapes, radius up to 400 px), one request at a time,
    through the surrogate service and through the plain path, with per-request
    latency and the surrogate's band error against the plain path."""
    import numpy as np
    import torch
    from paper_2006_10004_amd import nn, quality as Q, surrogate as S, synth

    dev = torch.device("cuda:0")
    rec = {"workload": "3x256x256 synthetic shape images (half 40-shape images, half crops of 1024x1024 "
                       "300-shape images), encoder-decoder 48-96-192-384, 4 bands x 3 + residual; "
                       "targets from the plain path dt 0.005, K 100, 150 iterations",
           "train_images": n_train, "test_images": test_images, "steps": steps, "batch": batch, "lr": lr,
           "lr_schedule": "linear warm-up over %d steps to lr, cosine decay to %g" % (S.LR_WARMUP, S.LR_FLOOR)}
    t0 = time.perf_counter()
    imgs = np.concatenate([S.make_training_images(n_train, 256, 20000 + seed),
                           S.make_training_images(test_images, 256, 90000 + seed)])
    f = torch.from_numpy(imgs).to(dev)
    rec["data_gen_s"] = time.perf_counter() - t0
    (bands, res), dt = S.timed(S.decompose_dataset, f)
    px = (n_train + test_images) * 256 * 256
    rec["plain_batch_256"] = {"images": n_train + test_images, "s": dt, "MPix_per_s": px / 1e6 / dt}
    print("bench: surrogate training data ready (%.1f s)" % dt, file=sys.stderr, flush=True)
    ftr, btr, rtr = f[:n_train], bands[:n_train], res[:n_train]
    fte, bte, rte = f[n_train:], bands[n_train:], res[n_train:]
    net = nn.Net(256, 256, batch, seed=seed)
    net.set_output_scale(S.output_scales(btr, rtr))
    net.set_loss_floor(S.LOSS_FLOOR)
    net.set_grad_clip(S.GRAD_CLIP)
    losses = []
    t1 = time.perf_counter()
    # the loss is read back every 25th step (the steps between only enqueue)
    for a in range(0, steps, 250):
        losses += S.train(net, ftr, btr, rtr, min(250, steps - a), batch,
                          lambda i, a=a: S.cosine_lr(a + i, steps, peak=lr), seed=seed + a, loss_every=25)
        print("bench: surrogate step %d loss %.4f" % (min(steps, a + 250), float(np.mean(losses[-2:]))),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tt = time.perf_counter() - t1
    rec["train"] = {"s": tt, "ms_per_step": tt * 1e3 / max(steps, 1), "loss_first25": losses[0] if losses else None,
                    "loss_last250": float(np.mean(losses[-10:])) if losses else None}
    out = torch.cat([net.forward(fte[i:i + batch].contiguous()) for i in range(0, test_images, batch)])
    rec["band_rel_l1"] = S.band_errors(out, bte, rte)
    pb, pr = S.split_output(out)
    rec["quality_256"] = Q.band_quality(pb, bte, pr, rte)
    rec["quality_256"]["definitions"] = ("PSNR with MAX_I = 1, SSIM (11x11 Gaussian window, sigma 1.5), sLMSE "
                                         "(16x16 patches, stride 8); per band over the held-out images")
    err = nn.tvspec_net_identity_error(fte.contiguous(), out).cpu().numpy()
    rec["identity_error"] = {"mean": float(err.mean()), "max": float(err.max())}
    # inference throughput (batch of 16 at 256^2): HIP events on the stream
    # the kernels run on, around back-to-back passes; the host clock around
    # the same kind of loop (launches included) is reported beside it
    x = fte[:batch].contiguous()
    o = net.forward(x)
    for _ in range(3):
        net.forward(x, o)
    reps = 20
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        net.forward(x, o)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    _, ti = S.timed(lambda: [net.forward(x, o) for _ in range(reps)])
    flops = S.conv_flops(256, 256) * batch
    achieved = flops / (ms / 1e3) / 1e12
    rec["inference_256"] = {"batch": batch, "ms": ms, "host_clock_ms": ti * 1e3 / reps,
                            "MPix_per_s": batch * 65536 / 1e6 / (ms / 1e3),
                            "channel_MPix_per_s": 3 * batch * 65536 / 1e6 / (ms / 1e3)}
    rec["roofline"] = {"kernel": "network forward (k_conv3x3, bf16 MFMA)", "bound": "mfma", "achieved": achieved,
                       "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / MFMA_BF16_PEAK_TFLOPS,
                       "flops_per_image": S.conv_flops(256, 256), "traffic": None}
    # serving with fallback on the held-out images
    svc = S.SurrogateService(net, threshold=1e-2, judge_every=8, max_judged_l1=SURROGATE_MAX_JUDGED_L1)
    _, ts = S.timed(lambda: [svc.decompose(fte[i:i + batch].contiguous()) for i in range(0, test_images, batch)])
    judged = svc.judged
    rec["service_256"] = {"threshold": 1e-2, "requests": test_images, "fallbacks": svc.fallbacks,
                          "judged": len(judged), "s": ts, "MPix_per_s": test_images * 65536 / 1e6 / ts,
                          "judged_all_bands_rel_l1": float(np.mean([j["all_bands"] for j in judged])) if judged
                          else None, "max_judged_all_bands_rel_l1": SURROGATE_MAX_JUDGED_L1,
                          "sizes": svc.size_info()}
    print("bench: surrogate 256x256 evaluation done", file=sys.stderr, flush=True)
    rec["megapixel"] = megapixel_serving(net, mega_sides, mega_requests, seed)
    net.close()
    return rec


def surrogate_forward_only(reps, batch=16, side=256, seed=11):
    """Forward passes of a freshly initialised network on one batch of
    `batch` 3 x side^2 shape images (dense convolutions cost the same for
    any weight values): the network's inference throughput and MFMA
    roofline alone, without training; the command to profile its kernels."""
    import torch
    from paper_2006_10004_amd import nn, surrogate as S

    dev = torch.device("cuda:0")
    net = nn.Net(side, side, batch, seed=seed)
    x = torch.from_numpy(S.make_images(batch, side, 70000 + seed)).to(dev)
    out = net.forward(x)
    for _ in range(3):
        net.forward(x, out)
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        net.forward(x, out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = S.conv_flops(side, side) * batch
    achieved = flops / (ms / 1e3) / 1e12
    net.close()
    return {"workload": "network forward, batch %d of 3x%dx%d" % (batch, side, side), "reps": reps, "ms": ms,
            "MPix_per_s": batch * side * side / 1e6 / (ms / 1e3),
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / MFMA_BF16_PEAK_TFLOPS, "flops_per_pass": flops}}


def surrogate_train_only(steps, batch=16, side=256, seed=11):
    """`steps` Adam steps (loss floor and gradient clipping as in training)
    on one batch of `batch` 3 x side^2 shape images with synthetic targets of
    the decomposition's shapes (kernel cost does not depend on the values):
    the training step's speed alone; the command to profile its kernels."""
    import numpy as np
    import torch
    from paper_2006_10004_amd import nn, surrogate as S

    dev = torch.device("cuda:0")
    net = nn.Net(side, side, batch, seed=seed)
    f = torch.from_numpy(S.make_images(batch, side, 80000 + seed)).to(dev)
    g = torch.Generator(device="cpu").manual_seed(seed)
    bands = (0.01 * torch.randn((batch, 4, 3, side, side), generator=g, dtype=torch.float64)).to(dev)
    res = f.double() - bands.sum(dim=1)
    net.set_output_scale(S.output_scales(bands, res))
    net.set_loss_floor(S.LOSS_FLOOR)
    net.set_grad_clip(S.GRAD_CLIP)
    for _ in range(3):
        net.train_step(f, bands, res, 1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        net.train_step(f, bands, res, 1e-3, sync=(i == steps - 1))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    net.close()
    flops = 3 * S.conv_flops(side, side) * batch  # forward, input and weight gradients
    return {"workload": "network training step, batch %d of 3x%dx%d" % (batch, side, side), "steps": steps,
            "ms_per_step": ms, "images_per_s": batch / (ms / 1e3),
            "conv_TFLOP_per_s": flops / (ms / 1e3) / 1e12}


def megapixel_serving(net, sides, n_req, seed):
    """Megapixel requests served one at a time (each waited for): through the
    surrogate service (identity-error fallback at 1e-2) and through the plain
    path with the flow the surrogate was trained on, on the same images."""
    import numpy as np
    import torch
    from paper_2006_10004_amd import nn, quality as Q, surrogate as S, synth

    dev = torch.device("cuda:0")
    p, scale = net.get_params(), net.output_scale
    svc = {}
    for side in sides:
        big = nn.Net(side, side, 1, seed=seed)
        big.set_params(p)
        big.set_output_scale(scale)
        svc[side] = S.SurrogateService(big, threshold=1e-2, judge_every=0)
    reqs = [(sides[i % len(sides)], 40000 + seed + i) for i in range(n_req)]
    lat_s, lat_p, outs = [], [], []
    num = {k: 0.0 for k in ("band1", "band2", "band3", "band4", "residual", "all_bands")}
    den = dict(num)
    ident, quals = [], []
    for side, s in [(sides[0], 1), (sides[-1], 2)]:           # warm both sizes
        fw = S.make_images(1, side, 50000 + s, spec=synth.megapixel_spec(side))
        svc[side].decompose(torch.from_numpy(fw).to(dev))
    for side, s in reqs:
        f = torch.from_numpy(S.make_images(1, side, s, spec=synth.megapixel_spec(side))).to(dev)
        r, t = S.timed(svc[side].decompose, f)
        lat_s.append(t * 1e3)
        ident.append(float(r["identity_error"][0]))
        (pb, pr), tp = S.timed(S.decompose_dataset, f)
        lat_p.append(tp * 1e3)
        for j in range(4):
            num["band%d" % (j + 1)] += float((r["bands"][0, j].double() - pb[0, j]).abs().sum())
            den["band%d" % (j + 1)] += float(pb[0, j].abs().sum())
        num["residual"] += float((r["residual"][0].double() - pr[0]).abs().sum())
        den["residual"] += float(pr[0].abs().sum())
        num["all_bands"] += float((r["bands"][0].double() - pb[0]).abs().sum())
        den["all_bands"] += float(pb[0].abs().sum())
        quals.append(Q.band_quality(r["bands"].double(), pb, r["residual"].double(), pr))
        print("bench: megapixel request %dx%d surrogate %.1f ms plain %.1f ms" % (side, side, lat_s[-1], tp * 1e3),
              file=sys.stderr, flush=True)
    mpix = sum(side * side for side, _ in reqs) / 1e6
    rec = {"workload": "3-channel shape images, 300 shapes, radius U[3,400], noise 0.02, sides %s alternating; "
                       "one request at a time" % list(sides),
           "requests": n_req,
           "surrogate": {"MPix_per_s": mpix / (sum(lat_s) / 1e3), "p50_ms": percentile(lat_s, 50),
                         "p99_ms": percentile(lat_s, 99),
                         "fallbacks": sum(v.fallbacks for v in svc.values()), "threshold": 1e-2},
           "plain": {"MPix_per_s": mpix / (sum(lat_p) / 1e3), "p50_ms": percentile(lat_p, 50),
                     "p99_ms": percentile(lat_p, 99), "flow": dict(S.FLOW)},
           "band_rel_l1": {k: num[k] / den[k] for k in num},
           "quality": {part: {m: float(np.mean([q[part][m] for q in quals])) for m in ("PSNR", "SSIM", "sLMSE")}
                       for part in quals[0]},
           "identity_error": {"mean": float(np.mean(ident)), "max": float(np.max(ident))}}
    rec["speedup"] = rec["surrogate"]["MPix_per_s"] / rec["plain"]["MPix_per_s"]
    # the plain path with the megapixel workload's own flow (dt 0.002, K 300,
    # 200 iterations, 4 dyadic bands), one request per side: its bands are
    # not the network's (other time samples), so this is a latency figure
    flow = dict(dt=0.002, K=300, iters=200, edges=[0, 1, 2, 4, 300])
    lat_m, mp_m = [], 0.0
    for side, s in [(side, 60000 + seed + i) for i, side in enumerate(sides)]:
        f = torch.from_numpy(S.make_images(1, side, s, spec=synth.megapixel_spec(side))).to(dev)
        _, tm = S.timed(S.decompose_dataset, f, flow)
        lat_m.append(tm * 1e3)
        mp_m += side * side / 1e6
        print("bench: megapixel plain path, its own flow, %dx%d: %.0f ms" % (side, side, tm * 1e3), file=sys.stderr,
              flush=True)
    rec["paper_context"] = dict(PAPER_1024_CONTEXT)
    pit = sum(3 * side * side * (flow["K"] + 1) * flow["iters"] for side in sides)
    rec["plain_megapixel_flow"] = {"flow": flow, "sides": list(sides), "ms": lat_m,
                                   "MPix_per_s": mp_m / (sum(lat_m) / 1e3),
                                   "alu_roofline": whole_job_alu(pit, sum(lat_m) / 1e3),
                                   "surrogate_speedup": rec["surrogate"]["MPix_per_s"] / (mp_m / (sum(lat_m) / 1e3))}
    for v in svc.values():
        v.net.close()
    return rec


def serving_bench(n_req, rate, burst, budget_gb, precision, seed=7, pool=4, fixed_requests=SERVING_FIXED_REQUESTS):
    """The serving workload through the server: first a burst of `burst`
    requests submitted at once (sustainable throughput), then n_req requests
    with Poisson arrivals at `rate` per second (0: 85% of the burst's
    request rate).  Inputs (a pool of `pool` images per side) and every
    request's outputs are resident in HBM before the timed region.  Latency
    is the server's own submission-to-completion time per request."""
    import threading

    import numpy as np
    import torch
    from paper_2006_10004_amd import synth, tvspec

    sv = SERVING
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    imgs = {s: [torch.from_numpy(synth.shapes_image(synth.serving_spec(s), 10000 * s + i)).to(dev)
                for i in range(pool)] for s in sv["sides"]}
    edges = tvspec.tvspec_dyadic_edges(sv["K"], sv["n_bands"])
    C, K = sv["C"], sv["K"]

    def make_jobs(n):
        sides = rng.choice(sv["sides"], size=n)
        jobs = []
        for i, s in enumerate(sides):
            s = int(s)
            out = {"bands": torch.empty((sv["n_bands"], C, s, s), dtype=torch.float64, device=dev),
                   "S": torch.empty((C, K), dtype=torch.float64, device=dev),
                   "residual": torch.empty((C, s, s), dtype=torch.float64, device=dev),
                   "stats": torch.empty((tvspec.TVSPEC_NSTATS,), dtype=torch.float64, device=dev)}
            jobs.append((s, imgs[s][i % pool], out))
        return jobs

    def run(srv, jobs, arrivals):
        """Submit job i at arrivals[i] seconds; collect completions."""
        done = {}
        tickets = [None] * len(jobs)
        t_sub = [0.0] * len(jobs)
        finished = threading.Event()

        def collect():
            while len(done) < len(jobs):
                progressed = False
                for i, t in enumerate(tickets):
                    if t is not None and i not in done:
                        r = srv.poll(t)
                        if r is not None:
                            done[i] = r
                            progressed = True
                if not progressed:
                    time.sleep(0.0005)
            finished.set()

        th = threading.Thread(target=collect, daemon=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th.start()
        for i, (s, f, out) in enumerate(jobs):
            while True:
                d = t0 + arrivals[i] - time.perf_counter()
                if d <= 0:
                    break
                time.sleep(min(d, 0.001))
            t_sub[i] = time.perf_counter() - t0
            tickets[i] = srv.submit(f, sv["dt"], K, sv["inner_iters"], edges, sync=False, out=out)[0]
        finished.wait(timeout=600)
        th.join(timeout=1)
        if len(done) < len(jobs):
            raise RuntimeError("serving bench: requests did not complete")
        lat = [done[i]["latency_ms"] for i in range(len(jobs))]
        end = max(t_sub[i] + lat[i] / 1e3 for i in range(len(jobs)))
        px = sum(s * s for s, _, _ in jobs)
        per_side = {}
        for side in sv["sides"]:
            ls = [lat[i] for i, (s, _, _) in enumerate(jobs) if s == side]
            if ls:
                per_side[str(side)] = {"n": len(ls), "p50_ms": percentile(ls, 50), "p99_ms": percentile(ls, 99)}
        worst = max(float(out["stats"][0]) for _, _, out in jobs)
        pit = sum(C * s * s * (K + 1) * sv["inner_iters"] for s, _, _ in jobs)
        return {"requests": len(jobs), "makespan_s": end, "MPix_per_s": px / 1e6 / end,
                "alu_roofline": whole_job_alu(pit, end, precision),
                "channel_MPix_per_s": C * px / 1e6 / end, "req_per_s": len(jobs) / end,
                "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                "mean_ms": float(np.mean(lat)), "queue_p99_ms": percentile([done[i]["queue_ms"] for i in done], 99),
                "per_side": per_side, "max_recon_err": worst}

    budget = int(budget_gb * (1 << 30))
    rec = {"workload": sv["workload"], "config": {k: v for k, v in sv.items() if k != "workload"},
           "precision": precision, "budget_GiB": budget_gb}
    with tvspec.Server(budget, precision=precision) as srv:
        # warm the buckets (graphs, and the autotuner's timed steps: 6
        # candidates x 3 steps) on one request of every side
        warm = [(s, imgs[s][0], None) for s in sv["sides"]]
        for s, f, _ in warm:
            srv.submit(f, sv["dt"], 20, sv["inner_iters"], [0, 20])
        while srv.info()["completed"] < len(warm):
            time.sleep(0.001)
        jobs = make_jobs(burst)
        sat = run(srv, jobs, [0.0] * burst)
        del jobs
        rec["saturated"] = sat
        print("bench: serving burst done (%.2f req/s)" % sat["req_per_s"], file=sys.stderr, flush=True)
        r = rate if rate > 0 else 0.85 * sat["req_per_s"]
        jobs = make_jobs(n_req)
        arrivals = np.cumsum(rng.exponential(1.0 / r, size=n_req))
        arrivals -= arrivals[0]
        rec["poisson"] = run(srv, jobs, list(arrivals))
        rec["poisson"]["rate_req_per_s"] = r
        del jobs
        print("bench: serving Poisson run done (p99 %.0f ms)" % rec["poisson"]["p99_ms"], file=sys.stderr,
              flush=True)
        if fixed_requests > 0:
            jobs = make_jobs(fixed_requests)
            arrivals = np.cumsum(rng.exponential(1.0 / SERVING_FIXED_RATE, size=fixed_requests))
            arrivals -= arrivals[0]
            rec["poisson_fixed_rate"] = run(srv, jobs, list(arrivals))
            rec["poisson_fixed_rate"]["rate_req_per_s"] = SERVING_FIXED_RATE
            del jobs
        info = srv.info()
    rec["server"] = {k: info[k] for k in ("max_in_flight", "graph_builds", "buckets", "steps", "replays", "peak_bytes")}
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="mixed", choices=["f32", "mixed", "f64"])
    ap.add_argument("--iters-per-launch", type=int, default=0)
    ap.add_argument("--latency-calls", type=int, default=20)
    ap.add_argument("--batch-images", type=int, default=256,
                    help="also time one batched call over this many 64x64 images (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests of the Poisson serving run (0 = skip the serving benchmark)")
    ap.add_argument("--serve-burst", type=int, default=64,
                    help="requests of the saturating burst that precedes it")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="Poisson arrival rate, requests/s (0 = 85%% of the burst's rate)")
    ap.add_argument("--serve-budget-gb", type=float, default=32.0)
    ap.add_argument("--serve-fixed-requests", type=int, default=SERVING_FIXED_REQUESTS,
                    help="requests of the Poisson run at a fixed %g requests/s (0 = skip)" % SERVING_FIXED_RATE)
    ap.add_argument("--pdhg-steps", type=int, default=3,
                    help="also time this many decompositions with the primal-dual solver (0 = skip)")
    ap.add_argument("--sur-train-images", type=int, default=8192,
                    help="training images of the learned surrogate (0 = skip the surrogate)")
    ap.add_argument("--sur-steps", type=int, default=16000, help="Adam steps of the surrogate's training")
    ap.add_argument("--sur-forward-only", type=int, default=0, metavar="N",
                    help="instead of the benchmark, time N forward passes of the surrogate network "
                         "(batch 16 of 3x256x256) and print that record")
    ap.add_argument("--sur-train-only", type=int, default=0, metavar="N",
                    help="instead of the benchmark, time N training steps of the surrogate network "
                         "(batch 16 of 3x256x256) and print that record")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-precisions", action="store_true",
                    help="skip timing the workload in the other two precision modes")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark, run 4 plain device copies of MIB MiB each "
                         "(reference dispatches for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU (images and channels are independent "
              "decompositions and would shard across GPUs without communication; one image "
              "is not split). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4,
                          "dispatches": 4}), flush=True)
        return

    if args.sur_forward_only > 0:
        print(json.dumps(surrogate_forward_only(args.sur_forward_only)), flush=True)
        return
    if args.sur_train_only > 0:
        print(json.dumps(surrogate_train_only(args.sur_train_only)), flush=True)
        return

    from paper_2006_10004_amd import synth, tvspec

    wl = dict(WORKLOAD)
    wl["iters_per_launch"] = args.iters_per_launch
    wl["precision"] = args.precision
    wl["warm_start"] = False
    dev = torch.device("cuda:0")
    spec = synth.IMAGE_512
    f_host = synth.shapes_image(spec, wl["seed"])
    f = torch.from_numpy(f_host).to(dev)
    edges = tvspec.tvspec_dyadic_edges(wl["K"], wl["n_bands"])
    kw = dict(tau=wl["tau"], precision=args.precision, iters_per_launch=args.iters_per_launch)
    stream = torch.cuda.current_stream(dev)

    def run(out=None):
        return tvspec.tvspec_decompose_dev(f, wl["dt"], wl["K"], wl["inner_iters"], edges, out=out,
                                           stream=stream, **kw)

    out = run()
    for _ in range(max(args.warmup - 1, 0)):
        run(out)
    torch.cuda.synchronize()
    print("bench: warmup done", file=sys.stderr, flush=True)

    # throughput: K back-to-back decompositions on one stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        run(out)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    ms_per_step = wall * 1e3 / args.steps
    stats = out["stats"].cpu().numpy()
    print("bench: timed %d steps, %.2f ms/step" % (args.steps, ms_per_step), file=sys.stderr, flush=True)

    # latency: each call waited for on its own (host wall clock)
    lat = []
    for _ in range(args.latency_calls):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run(out)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)

    px = wl["H"] * wl["W"] * wl["C"]
    rec = {
        "metric": "MPix/s spectral-TV decomposition (plain vs surrogate) + p50/p99 latency",
        "value": px / 1e6 / (ms_per_step / 1e3),
        "unit": "MPix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": wl,
        "path": "plain",
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99), "calls": len(lat),
                       "device_p50": percentile(step_ms, 50), "device_p99": percentile(step_ms, 99)},
        "report": {"recon_err": float(stats[0]), "mean_err": float(stats[1]), "nonfinite": float(stats[2])},
    }

    if not args.no_roofline:
        tvspec.tvspec_timing_enable(True)
        try:
            run(out)
            torch.cuda.synchronize()
            t = tvspec.tvspec_timing_read()
        finally:
            tvspec.tvspec_timing_enable(False)
        avg_ms = t["kernel_ms"] / t["launches"]
        rec["roofline"] = alu_roofline("k_chambolle_tile", t, ms_per_step, args.precision,
                                       FLOPS_PER_PIXEL_ITER, BYTES_PER_PIXEL_ITER[args.precision],
                                       measured_traffic(args.precision, args.iters_per_launch))
        print("bench: roofline pass done", file=sys.stderr, flush=True)

    if args.pdhg_steps > 0:
        rec["pdhg"] = pdhg_block(f, wl, edges, args.precision, args.pdhg_steps)
        print("bench: primal-dual pass done", file=sys.stderr, flush=True)

    if not args.no_precisions:
        rec["precisions"] = other_precisions(f, wl, edges, out)
        print("bench: other precision modes done", file=sys.stderr, flush=True)

    if args.batch_images > 0:
        rec["batch_64x64"] = batch_throughput(args.batch_images, args.precision)
        print("bench: batched 64x64 pass done", file=sys.stderr, flush=True)

    if args.serve_requests > 0:
        rec["serving"] = serving_bench(args.serve_requests, args.serve_rate, args.serve_burst,
                                       args.serve_budget_gb, args.precision,
                                       fixed_requests=args.serve_fixed_requests)
        print("bench: serving pass done", file=sys.stderr, flush=True)

    if args.sur_train_images > 0:
        rec["surrogate"] = surrogate_block(args.sur_train_images, args.sur_steps)
        print("bench: surrogate pass done", file=sys.stderr, flush=True)

    # the host entry point (host buffers, PCIe-inclusive), once, for reference
    t1 = time.perf_counter()
    tvspec.tvspec_decompose(f_host, wl["dt"], wl["K"], wl["inner_iters"], edges)
    rec["host_entry_ms"] = (time.perf_counter() - t1) * 1e3

    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on the same workload ...", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(f_host, wl)

    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
