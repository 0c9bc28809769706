"""GPU tests of the continuous-batching server (tvspec_server_* / submit /
poll / wait) through the C ABI.

Every request's results must equal, bit for bit, those of
tvspec_decompose_dev with the server's options: the kernels apply the same
per-pixel arithmetic whatever else shares a slot table, and every reduction
is per request in a fixed order.  So the tests compare exactly:
  alone (one request in flight at a time) == in a mix of sizes == direct,
and the oracle check of the direct path carries over (one oracle case here
as well, within the parity tolerances of the direct tests).
"""
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2006_10004_amd import synth  # noqa: E402

TOL_BANDS = 2e-4
TOL_S64 = 1e-6
WAIT_S = 120.0


@pytest.fixture(scope="module")
def tv():
    from paper_2006_10004_amd import tvspec
    return tvspec


def image(C, H, W, seed):
    spec = synth.ShapeSpec(H, W, C, 6, (synth.DISK, synth.RECT, synth.ELLIPSE), 3, max(H, W) / 5, 0.5, 0.02,
                           0.4)
    return synth.shapes_image(spec, seed)


# (C, H, W, dt, K, iters, edges) -- sizes over several tiles with ragged
# tails, different K per bucket, two requests sharing one bucket
MIX = [
    (1, 64, 64, 0.005, 12, 40, [0, 1, 2, 4, 12]),
    (3, 48, 80, 0.004, 9, 30, [0, 1, 3, 9]),
    (1, 64, 64, 0.003, 20, 40, [0, 2, 20]),
    (2, 97, 70, 0.005, 7, 25, [0, 1, 7]),
    (1, 130, 66, 0.006, 5, 40, [0, 5]),
]


def inputs(dev):
    return [torch.from_numpy(image(C, H, W, 100 + i)).to(dev) for i, (C, H, W, *_r) in enumerate(MIX)]


def direct(tv, fs, precision="mixed", warm=False):
    out = []
    for f, (C, H, W, dt, K, iters, edges) in zip(fs, MIX):
        out.append(tv.tvspec_decompose_dev(f, dt, K, iters, edges, precision=precision, warm_start=warm))
    torch.cuda.synchronize()
    return out


def wait_all(srv, tickets):
    """Poll until every ticket completes (bounded); returns their timings."""
    deadline = time.monotonic() + WAIT_S
    done = {}
    while len(done) < len(tickets):
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        assert time.monotonic() < deadline, "server did not finish within %.0f s" % WAIT_S
        time.sleep(0.0005)
    return [done[t] for t in tickets]


def run_mix(tv, fs, alone, budget=1 << 30, **opts):
    with tv.Server(budget, **opts) as srv:
        outs = []
        if alone:
            for f, (C, H, W, dt, K, iters, edges) in zip(fs, MIX):
                t, o = srv.submit(f, dt, K, iters, edges)
                wait_all(srv, [t])
                outs.append(o)
        else:
            ts = []
            for f, (C, H, W, dt, K, iters, edges) in zip(fs, MIX):
                t, o = srv.submit(f, dt, K, iters, edges)
                ts.append(t)
                outs.append(o)
            wait_all(srv, ts)
        info = srv.info()
    return outs, info


def assert_same(a, b):
    for k in ("bands", "S", "residual", "stats"):
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert x.shape == y.shape, k
        assert np.array_equal(x, y), (k, float(np.abs(x - y).max()))


def test_mix_equals_alone_equals_direct(tv):
    dev = torch.device("cuda:0")
    fs = inputs(dev)
    ref = direct(tv, fs)
    alone, info_a = run_mix(tv, fs, alone=True)
    mix, info_m = run_mix(tv, fs, alone=False)
    for i in range(len(MIX)):
        assert_same(alone[i], ref[i])
        assert_same(mix[i], ref[i])
    assert info_a["max_in_flight"] == 1
    assert info_m["max_in_flight"] >= 2, info_m
    assert info_m["buckets"] == 4
    assert info_m["completed"] == len(MIX) and info_m["used_bytes"] == 0
    assert info_m["graph_builds"] >= 1


@pytest.mark.parametrize("opts", [dict(use_graphs=False), dict(iters_per_launch=3),
                                  dict(precision="f64"), dict(precision="f32", iters_per_launch=16),
                                  dict(warm_start=True)],
                         ids=["no-graphs", "ipl3", "f64", "f32", "warm"])
def test_options_equal_direct(tv, opts):
    dev = torch.device("cuda:0")
    fs = inputs(dev)
    ref = direct(tv, fs, precision=opts.get("precision", "mixed"), warm=opts.get("warm_start", False))
    mix, _ = run_mix(tv, fs, alone=False, **opts)
    for i in range(len(MIX)):
        assert_same(mix[i], ref[i])


def test_tuned_multistep_replays_equal_direct(tv):
    """Flows long enough for the autotuner to time every (tile shape,
    blocking factor) candidate and then run several ROF solves per graph
    replay, with requests of different K sharing a bucket (so replays shrink
    to what the shortest request still needs): results equal the direct
    path's bit for bit."""
    dev = torch.device("cuda:0")
    cases = [(1, 64, 64, 0.005, 41, 30, [0, 1, 2, 4, 41]), (1, 64, 64, 0.004, 27, 30, [0, 3, 27]),
             (3, 48, 80, 0.005, 33, 20, [0, 1, 33])]
    fs = [torch.from_numpy(image(C, H, W, 300 + i)).to(dev) for i, (C, H, W, *_r) in enumerate(cases)]
    ref = [tv.tvspec_decompose_dev(f, dt, K, it, e) for f, (C, H, W, dt, K, it, e) in zip(fs, cases)]
    torch.cuda.synchronize()
    with tv.Server(1 << 30) as srv:
        ts, outs = [], []
        for f, (C, H, W, dt, K, it, e) in zip(fs, cases):
            t, o = srv.submit(f, dt, K, it, e)
            ts.append(t)
            outs.append(o)
        wait_all(srv, ts)
        info = srv.info()
    for a, b in zip(outs, ref):
        assert_same(a, b)
    # the two 64 x 64 requests share their bucket's 42 steps (more if the
    # second joins late); the other bucket takes 34; after each bucket's 18
    # timed single steps come runs of up to 4
    assert info["steps"] >= 42 + 34, info
    assert info["replays"] <= info["steps"] - 20, info


def test_budget_limits_admission(tv):
    """A pool that holds little more than the largest request's working
    state: admission waits for memory to free up, the pool's peak stays
    within the budget, and the results are the same; a request larger than
    the whole budget is refused with EBUSY."""
    from paper_2006_10004_amd import tvspec
    dev = torch.device("cuda:0")
    fs = inputs(dev)
    ref = direct(tv, fs)
    # working state of the largest request, as the header documents it (an
    # upper bound; admission uses the library's exact figure)
    need = 0
    for (C, H, W, dt, K, iters, edges) in MIX:
        n = C * H * W
        nblk = min(1024, (H * W + 255) // 256)
        need = max(need, n * (4 * 8 + 2 * 4 + 24) + C * K * 8 * nblk + 4096 * 8)
    budget = max(need, 1 << 20)
    mix, info = run_mix(tv, fs, alone=False, budget=budget)
    for i in range(len(MIX)):
        assert_same(mix[i], ref[i])
    assert info["peak_bytes"] <= info["budget_bytes"]
    assert info["max_in_flight"] < len(MIX)
    with pytest.raises(tvspec.TvspecError) as ei:
        with tv.Server(1 << 20) as srv:
            f = torch.from_numpy(image(3, 256, 256, 1)).to(dev)
            srv.submit(f, 0.005, 10, 10, [0, 10])
    assert ei.value.code == tvspec.TVSPEC_EBUSY


def test_request_joins_while_others_run(tv):
    """Continuous batching: short requests submitted while a long one is on
    the device are admitted at once and complete before it does."""
    dev = torch.device("cuda:0")
    long_f = torch.from_numpy(image(1, 64, 64, 7)).to(dev)
    short_f = [torch.from_numpy(image(1, 64, 64, 8 + i)).to(dev) for i in range(3)]
    with tv.Server(1 << 30, iters_per_launch=8) as srv:
        t_long, o_long = srv.submit(long_f, 0.001, 3000, 64, [0, 1, 3000])
        deadline = time.monotonic() + WAIT_S
        while srv.info()["admitted"] < 1:
            assert time.monotonic() < deadline
            time.sleep(0.0005)
        time.sleep(0.01)
        ts, os_ = [], []
        for f in short_f:
            t, o = srv.submit(f, 0.005, 4, 20, [0, 4])
            ts.append(t)
            os_.append(o)
        res = wait_all(srv, ts)
        assert srv.poll(t_long) is None, "the long request finished before the short ones"
        info = srv.info()
        assert info["max_in_flight"] >= 2
        wait_all(srv, [t_long])
    for r in res:
        assert r["queue_ms"] < 1000.0
    refs = [tv.tvspec_decompose_dev(f, 0.005, 4, 20, [0, 4]) for f in short_f]
    ref_long = tv.tvspec_decompose_dev(long_f, 0.001, 3000, 64, [0, 1, 3000])
    torch.cuda.synchronize()
    for o, r in zip(os_, refs):
        assert_same(o, r)
    assert_same(o_long, ref_long)


def test_many_requests_reuse_slots_and_memory(tv):
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(3)
    sizes = [(1, 32, 32), (1, 40, 56), (3, 33, 33)]
    fs = [torch.from_numpy(image(*sizes[i % 3], 200 + i)).to(dev) for i in range(6)]
    jobs = []
    for i in range(48):
        K = int(rng.integers(1, 9))
        jobs.append((i % 6, K, [0, K]))
    # a budget of a few requests: admission waits for memory to free up
    budget = 3 * (3 * 33 * 33 * 64 + 9 * 3 * 8 * 5 + 8192)
    budget = max(budget, 1 << 20)
    with tv.Server(budget) as srv:
        ts, outs = [], []
        for fi, K, e in jobs:
            t, o = srv.submit(fs[fi], 0.004, K, 15, e)
            ts.append(t)
            outs.append(o)
        wait_all(srv, ts)
        info = srv.info()
    assert info["completed"] == 48 and info["admitted"] == 48 and info["used_bytes"] == 0
    for j in (0, 7, 20, 33, 47):
        fi, K, e = jobs[j]
        r = tv.tvspec_decompose_dev(fs[fi], 0.004, K, 15, e)
        torch.cuda.synchronize()
        assert_same(outs[j], r)


def test_run_cap_admits_saturating_requests_one_at_a_time(tv):
    """Three 3 x 2048 x 2048 requests each fill the device several times
    over (12288 workgroups per launch): the bucket runs them one at a time
    (peak one of them in flight) while a small request submitted after them
    is not held back; every result equals the direct path's."""
    dev = torch.device("cuda:0")
    big = [torch.from_numpy(image(3, 2048, 2048, 300 + i)).to(dev) for i in range(3)]
    small = torch.from_numpy(image(1, 64, 64, 310)).to(dev)
    with tv.Server(1 << 34) as srv:
        ts, outs = [], []
        for f in big:  # ~40 ms each on the device
            t, o = srv.submit(f, 0.004, 20, 40, [0, 1, 20])
            ts.append(t)
            outs.append(o)
        t_small, o_small = srv.submit(small, 0.004, 3, 10, [0, 1, 3])
        res = wait_all(srv, ts + [t_small])
        info = srv.info()
    assert info["completed"] == 4 and info["max_in_flight"] == 2, info
    # the small request was admitted while the first large one ran
    assert res[3]["queue_ms"] < res[1]["queue_ms"]
    for f, o in zip(big, outs):
        assert_same(o, tv.tvspec_decompose_dev(f, 0.004, 20, 40, [0, 1, 20]))
    assert_same(o_small, tv.tvspec_decompose_dev(small, 0.004, 3, 10, [0, 1, 3]))
    torch.cuda.synchronize()


def test_server_against_oracle(tv, orc):
    dev = torch.device("cuda:0")
    f = synth.shapes_image(synth.SMALL_64, 0)
    edges = [0, 1, 2, 4, 60]
    with tv.Server(1 << 28) as srv:
        t, o = srv.submit(torch.from_numpy(f).to(dev), 0.005, 60, 200, edges)
        wait_all(srv, [t])
    ref = orc.decompose(f, dt=0.005, K=60, iters=200, edges=edges)
    b = o["bands"].cpu().numpy()
    assert np.abs(b - ref["bands"]).max() <= TOL_BANDS
    assert np.abs(o["residual"].cpu().numpy() - ref["residual"]).max() <= TOL_BANDS
    S = o["S"].cpu().numpy()
    assert np.abs(S - ref["S"]).max() / np.abs(ref["S"]).max() <= TOL_S64
    st = o["stats"].cpu().numpy()
    assert st[0] <= 1e-12 and st[2] == 0


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_serving_size_request_against_oracle(tv, orc):
    """One request of the serving workload's largest size (3 x 1024 x 1024,
    40 shapes, dt 0.005, K 100, 150 iterations, 4 dyadic bands) through the
    server, sharing it with a smaller request, against the oracle's full
    run."""
    dev = torch.device("cuda:0")
    f = synth.shapes_image(synth.serving_spec(1024), 4242)
    small = torch.from_numpy(image(3, 128, 128, 4243)).to(dev)
    edges = [0, 1, 2, 4, 100]
    print("serving-size request: 3x1024x1024, K 100, 150 iterations", flush=True)
    with tv.Server(4 << 30) as srv:
        t, o = srv.submit(torch.from_numpy(f).to(dev), 0.005, 100, 150, edges)
        t2, _ = srv.submit(small, 0.005, 100, 150, edges)
        wait_all(srv, [t, t2])
    ref = orc.decompose(f, dt=0.005, K=100, iters=150, edges=edges)
    assert np.abs(o["bands"].cpu().numpy() - ref["bands"]).max() <= TOL_BANDS
    assert np.abs(o["residual"].cpu().numpy() - ref["residual"]).max() <= TOL_BANDS
    S = o["S"].cpu().numpy()
    assert np.abs(S - ref["S"]).max() / np.abs(ref["S"]).max() <= TOL_S64
    st = o["stats"].cpu().numpy()
    assert st[0] <= 1e-12 and st[1] <= 1e-12 and st[2] == 0


def test_invalid_requests(tv):
    from paper_2006_10004_amd import tvspec
    dev = torch.device("cuda:0")
    f = torch.from_numpy(image(1, 32, 32, 1)).to(dev)
    with tv.Server(1 << 24) as srv:
        for args in [(0.0, 5, 10, [0, 5]), (0.01, 0, 10, [0, 1]), (0.01, 5, 0, [0, 5]),
                     (0.01, 5, 10, [0, 3, 2, 5]), (0.01, 5, 10, [1, 5])]:
            with pytest.raises(tvspec.TvspecError) as ei:
                srv.submit(f, *args)
            assert ei.value.code == tvspec.TVSPEC_EINVAL
        with pytest.raises(tvspec.TvspecError) as ei:
            srv.poll(12345)
        assert ei.value.code == tvspec.TVSPEC_EINVAL
        t, _ = srv.submit(f, 0.01, 3, 10, [0, 3])
        wait_all(srv, [t])
        with pytest.raises(tvspec.TvspecError):
            srv.poll(t)  # retired
