"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/tvspec.h declares, and rejects invalid arguments before any device
work; the product path does not reach the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tvspec.h")
LIB = os.path.join(ROOT, "paper_2006_10004_amd", "libtvspec.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tvspec_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def tv():
    from paper_2006_10004_amd import tvspec
    return tvspec


def test_header_symbols_exported():
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header(tv):
    assert sorted(tv.EXPORTS) == declared()
    for n in declared():
        assert callable(getattr(tv, n))


NN_HEADER = os.path.join(ROOT, "include", "tvspec_nn.h")


def test_nn_header_symbols_exported_and_bound():
    text = re.sub(r"/\*.*?\*/", "", open(NN_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(tvspec_(?:nn|net)_\w+)\s*\(", text)))
    assert len(names) >= 10
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    from paper_2006_10004_amd import nn
    assert sorted(nn.EXPORTS) == names
    for n in names:
        assert callable(getattr(nn, n))


def test_nn_entry_validation():
    """Shape checks of the surrogate's entry points run before device work."""
    lib = ctypes.CDLL(LIB)
    vp, ci = ctypes.c_void_p, ctypes.c_int
    lib.tvspec_nn_conv3x3.argtypes = [vp, ci, ci, ci, ci, vp, vp, ci, ci, vp, ci, vp]
    fake = vp(0x1000)
    assert lib.tvspec_nn_conv3x3(fake, 1, 4, 4, 6, fake, None, 16, 0, fake, 0, None) == -1   # Cin % 8
    assert lib.tvspec_nn_conv3x3(fake, 1, 4, 4, 8, fake, None, 24, 0, fake, 0, None) == -1   # Cout % 16
    assert lib.tvspec_nn_conv3x3(fake, 0, 4, 4, 8, fake, None, 16, 0, fake, 0, None) == -1
    lib.tvspec_net_create.argtypes = [ci, ci, ci, ctypes.c_ulonglong, ctypes.POINTER(vp)]
    h = vp()
    for H, W, B in [(20, 32, 1), (32, 12, 1), (32, 32, 0)]:
        assert lib.tvspec_net_create(H, W, B, 0, ctypes.byref(h)) == -1
    lib.tvspec_net_destroy.argtypes = [vp]
    assert lib.tvspec_net_destroy(None) == 0
    cf = ctypes.c_float
    lib.tvspec_net_set_grad_clip.argtypes = [vp, cf]
    lib.tvspec_net_set_loss_floor.argtypes = [vp, cf]
    assert lib.tvspec_net_set_grad_clip(None, 2.0) == -1
    assert lib.tvspec_net_set_loss_floor(None, 0.1) == -1
    lib.tvspec_net_grad_stats.argtypes = [vp, vp, vp, vp]
    assert lib.tvspec_net_grad_stats(None, fake, fake, fake) == -1
    lib.tvspec_net_forward_checked.argtypes = [vp, vp, ci, vp, vp, vp]
    assert lib.tvspec_net_forward_checked(None, fake, 1, fake, None, None) == -1


def test_version(tv):
    assert "gfx950" in tv.tvspec_version()


def test_dyadic_edges(tv):
    assert tv.tvspec_dyadic_edges(50, 6) == [0, 1, 2, 4, 8, 16, 50]
    assert tv.tvspec_dyadic_edges(60, 4) == [0, 1, 2, 4, 60]
    assert tv.tvspec_dyadic_edges(200, 8) == [0, 1, 2, 4, 8, 16, 32, 64, 200]
    assert tv.tvspec_dyadic_edges(5, 1) == [0, 5]
    for K, B in ((4, 5), (0, 2), (8, 0)):
        with pytest.raises(tv.TvspecError) as ei:
            tv.tvspec_dyadic_edges(K, B)
        assert ei.value.code == tv.TVSPEC_EINVAL


BAD = [
    dict(H=1), dict(W=1), dict(C=0), dict(dt=0.0), dict(dt=float("nan")), dict(dt=float("inf")),
    dict(K=0), dict(iters=0), dict(edges=[0, 2, 2, 4]), dict(edges=[1, 4]), dict(edges=[0, 3]),
    dict(nb=0), dict(nb=5), dict(H=1 << 16, W=1 << 16),
]


@pytest.mark.parametrize("bad", BAD)
def test_host_entry_validation(bad):
    """Invalid arguments return TVSPEC_EINVAL before any device call (so this
    runs on a machine without a GPU)."""
    lib = ctypes.CDLL(LIB)
    a = dict(H=4, W=5, C=1, dt=0.1, K=4, iters=3, edges=[0, 1, 4], nb=None)
    a.update(bad)
    e = np.array(a["edges"], dtype=np.int32)
    nb = len(e) - 1 if a["nb"] is None else a["nb"]
    f = np.zeros(16, np.float32)
    out = np.zeros(64, np.float64)
    lib.tvspec_decompose.restype = ctypes.c_int
    rc = lib.tvspec_decompose(f.ctypes.data_as(ctypes.c_void_p), a["H"], a["W"], a["C"],
                              ctypes.c_double(a["dt"]), a["K"], a["iters"],
                              e.ctypes.data_as(ctypes.c_void_p), nb,
                              out.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p),
                              out.ctypes.data_as(ctypes.c_void_p))
    assert rc == -1


def test_host_entry_null_pointer_and_nonfinite(tv):
    lib = ctypes.CDLL(LIB)
    e = np.array([0, 2], dtype=np.int32)
    out = np.zeros(64, np.float64)
    rc = lib.tvspec_decompose(None, 3, 3, 1, ctypes.c_double(0.1), 2, 3, e.ctypes.data_as(ctypes.c_void_p), 1,
                              out.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p),
                              out.ctypes.data_as(ctypes.c_void_p))
    assert rc == -1
    f = np.zeros((3, 3), np.float32)
    f[1, 1] = np.inf
    with pytest.raises(tv.TvspecError) as ei:
        tv.tvspec_decompose(f, 0.1, 2, 3, [0, 2])
    assert ei.value.code == tv.TVSPEC_ENUMERIC
    assert "NaN" in tv.tvspec_last_error() or "infinity" in tv.tvspec_last_error()


def test_device_entry_validation_options():
    """Option checks of the device entry point also run before device work."""
    lib = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    lib.tvspec_decompose_dev.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, vp, vp, vp, vp,
                                         ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    e = np.array([0, 4], dtype=np.int32)
    fake = vp(0x1000)  # never dereferenced: validation fails first
    base = dict(tau=0.248, warm=1, prec=0, ipl=0)
    for bad in (dict(tau=0.0), dict(tau=0.26), dict(warm=2), dict(prec=3), dict(prec=-1), dict(ipl=-1),
                dict(ipl=17), dict(prec=1, ipl=9), dict(prec=2, ipl=9)):
        a = dict(base)
        a.update(bad)
        rc = lib.tvspec_decompose_dev(fake, 8, 8, 1, 0.01, 4, 5, e.ctypes.data_as(vp), 1, fake, fake, fake, fake,
                                      a["tau"], a["warm"], a["prec"], a["ipl"], None)
        assert rc == -1, bad
    rc = lib.tvspec_decompose_dev(fake, 8, 8, 1, 0.01, 4, 5, e.ctypes.data_as(vp), 1, fake, fake, fake, None,
                                  0.248, 1, 0, 0, None)
    assert rc == -1


def test_pdhg_entry_validation():
    """The primal-dual entry point checks its steps before any device work."""
    lib = ctypes.CDLL(LIB)
    vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.tvspec_decompose_pdhg_dev.argtypes = [vp, ci, ci, ci, cd, ci, ci, vp, ci, vp, vp, vp, vp, cd, cd, ci, ci,
                                              ci, vp]
    e = np.array([0, 4], dtype=np.int32)
    fake = vp(0x1000)  # never dereferenced: validation fails first
    for tau, sigma in [(0.5, 0.5), (-0.1, 0.2), (0.2, -0.1), (0.0, 0.3), (float("inf"), 0.1)]:
        rc = lib.tvspec_decompose_pdhg_dev(fake, 8, 8, 1, 0.01, 4, 5, e.ctypes.data_as(vp), 1, fake, fake, fake,
                                           fake, tau, sigma, 0, 2, 0, None)
        assert rc == -1, (tau, sigma)
    rc = lib.tvspec_decompose_pdhg_dev(fake, 8, 8, 1, 0.01, 4, 5, e.ctypes.data_as(vp), 1, fake, fake, fake,
                                       fake, 0.0, 0.0, 0, 7, 0, None)
    assert rc == -1  # bad precision


def test_server_entry_validation():
    """Server entry points reject bad options and null handles before any
    device work."""
    lib = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    lib.tvspec_server_create.argtypes = [ctypes.c_size_t, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    h = vp()
    good = dict(budget=1 << 24, tau=0.248, warm=0, prec=2, ipl=0, graphs=1)
    for bad in (dict(budget=1000), dict(tau=0.3), dict(warm=3), dict(prec=5), dict(ipl=9), dict(graphs=2)):
        a = dict(good)
        a.update(bad)
        rc = lib.tvspec_server_create(a["budget"], a["tau"], a["warm"], a["prec"], a["ipl"], a["graphs"],
                                      ctypes.byref(h))
        assert rc == -1, bad
        assert h.value is None
    rc = lib.tvspec_server_create(1 << 24, 0.248, 0, 2, 0, 1, None)
    assert rc == -1
    lib.tvspec_submit.argtypes = [vp, vp, vp]
    assert lib.tvspec_submit(None, None, None) == -1
    lib.tvspec_poll.argtypes = [vp, ctypes.c_ulonglong, vp]
    assert lib.tvspec_poll(None, 1, None) == -1
    lib.tvspec_wait.argtypes = [vp, ctypes.c_ulonglong, vp]
    assert lib.tvspec_wait(None, 1, None) == -1
    lib.tvspec_server_info.argtypes = [vp, vp]
    assert lib.tvspec_server_info(None, None) == -1
    lib.tvspec_server_destroy.argtypes = [vp]
    assert lib.tvspec_server_destroy(None) == 0


def test_server_structs_match_header(tv):
    """The binding's ctypes structures have the header's field order."""
    text = open(HEADER).read()
    for name, cls in (("tvspec_request", tv._Request), ("tvspec_result", tv._Result),
                      ("tvspec_server_stats", tv._ServerStats), ("tvspec_args", tv._Args),
                      ("tvspec_options", tv._Options), ("tvspec_report", tv._Report)):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, flags=re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = re.findall(r"[\s\*]([A-Za-z_][A-Za-z_0-9]*)\s*(?=[,;])", body)
        assert fields == [f for f, _ in cls._fields_], (name, fields)


def test_ex_default_options(tv):
    o = tv.tvspec_default_options()
    assert o["solver"] == tv.TVSPEC_SOLVER_CHAMBOLLE and o["tau"] == 0.0 and o["warm_start"] == 0
    assert o["precision"] == tv.TVSPEC_PRECISION_MIXED and o["device_ptrs"] == 0 and o["stream"] is None
    assert o["tile_shape"] == tv.TVSPEC_TILE_SQUARE


EX_BAD = [
    (dict(solver=2), "solver"), (dict(device_ptrs=2), "device_ptrs"), (dict(tau=0.3), "tau"),
    (dict(solver=1, tau=0.5, sigma=0.5), "PDHG"), (dict(precision=4), "precision"),
    (dict(iters_per_launch=9), "iters_per_launch"), (dict(H=1), "H and W"), (dict(K=0), "K"),
    (dict(device_ptrs=1, stats=None), "null"), (dict(f=None), "null"), (dict(tile_shape=2), "tile_shape"),
    (dict(tile_shape=1, solver=1), "narrow"), (dict(tile_shape=1, precision=0, iters_per_launch=16), "narrow"),
]


@pytest.mark.parametrize("bad,msg", EX_BAD)
def test_ex_entry_validation_without_a_device(tv, bad, msg):
    """tvspec_decompose_ex rejects bad arguments and options with
    TVSPEC_EINVAL before any device work (host buffers stand in for device
    ones; none is touched)."""
    lib = ctypes.CDLL(LIB)
    lib.tvspec_decompose_ex.argtypes = [ctypes.POINTER(tv._Args), ctypes.POINTER(tv._Options),
                                        ctypes.POINTER(tv._Report)]
    lib.tvspec_last_error.restype = ctypes.c_char_p
    buf = np.zeros(256, np.float64)
    e = np.array([0, 1, 4], dtype=np.int32)
    a = dict(f=buf.ctypes.data, H=4, W=5, C=1, dt=0.1, K=4, iters=3, stats=buf.ctypes.data)
    o = tv._Options()
    lib_o = ctypes.CDLL(LIB)
    lib_o.tvspec_default_options(ctypes.byref(o))
    for k, v in bad.items():
        if k in a:
            a[k] = v
        else:
            setattr(o, k, v)
    args = tv._Args(a["f"], a["H"], a["W"], a["C"], a["dt"], a["K"], a["iters"], e.ctypes.data, 2,
                    buf.ctypes.data, buf.ctypes.data, buf.ctypes.data, a["stats"])
    rep = tv._Report()
    assert lib.tvspec_decompose_ex(ctypes.byref(args), ctypes.byref(o), ctypes.byref(rep)) == -1
    assert msg in lib.tvspec_last_error().decode()
    assert lib.tvspec_decompose_ex(None, None, None) == -1


def test_ex_host_nonfinite_before_device_work(tv):
    f = np.zeros((3, 4), np.float32)
    f[2, 1] = np.nan
    with pytest.raises(tv.TvspecError) as ei:
        tv.tvspec_decompose_ex(f, 0.1, 2, 3, [0, 2])
    assert ei.value.code == tv.TVSPEC_ENUMERIC


def test_noalloc_entry_rejects_oversize_without_a_device():
    """The allocation-free entry point checks its scratch need against its
    fixed array before any device work (host buffers stand in for device
    ones; none is touched)."""
    lib = ctypes.CDLL(LIB)
    vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.tvspec_decompose_noalloc_dev.argtypes = [vp, ci, ci, ci, cd, ci, ci, vp, ci, vp, vp, vp, vp, cd, ci, ci,
                                                 ci, vp]
    lib.tvspec_last_error.restype = ctypes.c_char_p
    e = np.array([0, 4], dtype=np.int32)
    fake = vp(0x1000)
    rc = lib.tvspec_decompose_noalloc_dev(fake, 1024, 1024, 3, 0.01, 4, 5, e.ctypes.data_as(vp), 1, fake, fake,
                                          fake, fake, 0.248, 0, 2, 0, None)
    assert rc == -1 and b"bytes of scratch" in lib.tvspec_last_error()
    many = np.arange(66, dtype=np.int32)
    rc = lib.tvspec_decompose_noalloc_dev(fake, 8, 8, 1, 0.01, 65, 5, many.ctypes.data_as(vp), 65, fake, fake,
                                          fake, fake, 0.248, 0, 2, 0, None)
    assert rc == -1 and b"64 bands" in lib.tvspec_last_error()


def test_product_path_never_reaches_the_oracle():
    """No module of the package, nor the HIP source, imports or links the
    oracle; there is no CPU fallback."""
    pkg = os.path.join(ROOT, "paper_2006_10004_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle", text, flags=re.M), fn
                assert "liboracle" not in text and "orc_" not in text, fn


BATCH_BAD = [
    (dict(B=0), "B must be >= 1"),
    (dict(B=-3), "B must be >= 1"),
    (dict(B=2, C=40000), "B*C"),
    (dict(H=1), "H and W"),
    (dict(iters=0), None),
    (dict(K1=0), "image 1"),
    (dict(dt1=float("nan")), "image 1"),
]


@pytest.mark.parametrize("bad,msg", BATCH_BAD)
def test_batch_entry_validation_without_a_device(bad, msg):
    """The batched entry rejects an empty batch, oversize batches and any
    image's invalid parameters with TVSPEC_EINVAL before it touches a
    pointer or the device (host buffers stand in for device ones here)."""
    lib = ctypes.CDLL(LIB)
    a = dict(B=2, H=4, W=5, C=1, iters=3, K1=4, dt1=0.1)
    a.update(bad)
    nb = max(a["B"], 2)
    dt = np.array([0.1, a["dt1"]] + [0.1] * (nb - 2), dtype=np.float64)
    K = np.array([4, a["K1"]] + [4] * (nb - 2), dtype=np.int32)
    n_bands = np.ones(nb, dtype=np.int32)
    edges = np.array([x for k in K for x in (0, k)], dtype=np.int32)
    buf = np.zeros(64, np.float64)
    p = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    lib.tvspec_decompose_batch_dev.restype = ctypes.c_int
    lib.tvspec_last_error.restype = ctypes.c_char_p
    rc = lib.tvspec_decompose_batch_dev(p(buf), a["B"], a["H"], a["W"], a["C"], a["iters"], p(dt), p(K), p(edges),
                                        p(n_bands), p(buf), p(buf), p(buf), p(buf), ctypes.c_double(0.248), 0, 2, 0,
                                        None)
    assert rc == -1
    if msg is not None:
        assert msg in lib.tvspec_last_error().decode()


@pytest.mark.parametrize("module", ["tvspec", "nn"])
def test_bindings_fail_loudly_without_the_library(tmp_path, module):
    """A copy of the package without libtvspec.so: importing a binding raises
    (there is no CPU path to fall back on)."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_2006_10004_amd"
    pkg.mkdir()
    for fn in os.listdir(os.path.join(ROOT, "paper_2006_10004_amd")):
        if fn.endswith(".py"):
            shutil.copy(os.path.join(ROOT, "paper_2006_10004_amd", fn), pkg / fn)
    r = subprocess.run([sys.executable, "-c", "import paper_2006_10004_amd.%s" % module], cwd=str(tmp_path),
                       env=dict(os.environ, PYTHONPATH=str(tmp_path)), capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "is not built" in r.stderr


def test_server_keeps_tensors_of_failed_tickets_until_close(tv, monkeypatch):
    """A ticket that fails (the server failed, e.g. an allocation error) keeps
    its tensors alive until close() has destroyed the server, because work
    enqueued before the failure may still use them; completed tickets drop
    theirs at once.  Bookkeeping only: the C calls are stubbed, no device."""
    srv = object.__new__(tv.Server)
    srv._h, srv._live, srv._graveyard = "handle", {}, []
    calls = []

    def poll(h, t):
        if t == 2:
            raise tv.TvspecError(tv.TVSPEC_EDEVICE, "server failed")
        return {"queue_ms": 0.0, "latency_ms": 1.0}

    def wait(h, t):
        raise tv.TvspecError(tv.TVSPEC_ENOMEM, "server failed")

    monkeypatch.setattr(tv, "tvspec_poll", poll)
    monkeypatch.setattr(tv, "tvspec_wait", wait)
    monkeypatch.setattr(tv, "tvspec_server_destroy", lambda h: calls.append(h))
    for t in (1, 2, 3):
        srv._live[t] = ("f%d" % t, {"out": t})
    assert srv.poll(1) == {"queue_ms": 0.0, "latency_ms": 1.0}
    assert 1 not in srv._live and srv._graveyard == []
    with pytest.raises(tv.TvspecError):
        srv.poll(2)
    with pytest.raises(tv.TvspecError):
        srv.wait(3)
    assert srv._live == {} and srv._graveyard == [("f2", {"out": 2}), ("f3", {"out": 3})]
    srv.close()
    assert calls == ["handle"] and srv._graveyard == [] and srv._h is None
