"""Host-side behaviour of bench.py that needs no GPU: one GPU only, and the
HBM-traffic record is read only for the kernel source it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_touching_a_device():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_tied_to_the_kernel_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    rec = json.loads(open(bench.TRAFFIC_RECORD).read().split("```json\n")[1].split("\n```")[0])
    assert rec["traffic_bytes_per_launch"] > 0
    # another source: the record no longer applies, traffic is reported as null
    other = tmp_path / "tile_kernels.h"
    other.write_text(open(bench.KERNEL_SOURCE).read() + "\n// edited\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(other))
    assert bench.measured_traffic("mixed", 0) is None
    assert bench.measured_traffic("mixed", 0, bench.PDHG_TRAFFIC_RECORD) is None


def test_primal_dual_traffic_record():
    sys.path.insert(0, ROOT)
    import bench
    rec = json.loads(open(bench.PDHG_TRAFFIC_RECORD).read().split("```json\n")[1].split("\n```")[0])
    # the writes are the four float64 planes x, xbar, yx, yy of 512 x 512
    assert rec["write_kib_per_dispatch"] == 4 * 512 * 512 * 8 / 1024
    want = (rec["fetch_kib_per_dispatch"] * rec["fetch_scale"] + rec["write_kib_per_dispatch"] * rec["write_scale"]) * 1024
    assert abs(rec["traffic_bytes_per_launch"] - want) < 1024
    import hashlib
    sha = hashlib.sha256(open(bench.KERNEL_SOURCE, "rb").read()).hexdigest()
    expect = rec["traffic_bytes_per_launch"] if rec["source_sha256"] == sha else None
    assert bench.measured_traffic("mixed", 0, bench.PDHG_TRAFFIC_RECORD) == expect
    assert bench.measured_traffic("f32", 0, bench.PDHG_TRAFFIC_RECORD) is None


def test_alu_roofline_record():
    """The roofline of a blocked tile kernel: algorithmic flops per launch
    over the average launch, against the mode's vector peak; the HBM rate
    only from counter bytes, and null without them."""
    sys.path.insert(0, ROOT)
    import bench
    t = {"kernel_ms": 10.0, "launches": 1000, "pixel_iters": 1000 * 2_000_000}
    r = bench.alu_roofline("k", t, 20.0, "mixed", 18, 40, None)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert abs(r["achieved"] - 18 * 2e6 / 10e-6 / 1e12) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 78.6) < 1e-12
    assert r["traffic"] is None and r["hbm_GBps"] is None
    assert abs(r["effective_GBps"] - 40 * 2e6 / 10e-6 / 1e9) < 1e-6
    r = bench.alu_roofline("k", t, 20.0, "f32", 18, 24, 10_000_000)
    assert r["peak"] == 157.3 and abs(r["hbm_GBps"] - 1000.0) < 1e-9


def test_cpu_baseline_reports_all_threads_and_one_thread():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2006_10004_amd import synth
    f = synth.shapes_image(synth.ShapeSpec(32, 40, 1), 3)
    wl = dict(H=32, W=40, C=1, dt=0.01, K=6, inner_iters=20, n_bands=3, tau=0.248)
    rec = bench.cpu_baseline(f, wl, one_thread_steps=2, others=False)
    assert rec["kind"] == "oracle" and rec["unit"] == "MPix/s"
    assert rec["value"] > 0 and rec["cores"] >= 1
    assert "7 ROF solves x 20 iterations" in rec["sample"]
    one = rec["one_thread"]
    assert one["cores"] == 1 and one["value"] > 0
    assert "3 ROF solves" in one["sample"]


def test_oracle_on_the_other_workloads():
    """The 64x64 workload in full and the megapixel flow per solve, scaled
    to its 301 solves."""
    sys.path.insert(0, ROOT)
    import bench
    rec = bench.oracle_other_workloads(mega_steps=1)
    small, mega = rec["64x64"], rec["3x1024x1024"]
    assert small["unit"] == "MPix/s" and abs(small["value"] - 64 * 64 / 1e6 / small["seconds"]) < 1e-12
    assert "61 ROF solves x 200" in small["sample"]
    assert abs(mega["value"] - 1024 * 1024 / 1e6 / mega["seconds_full_estimate"]) < 1e-12
    assert "2 ROF solves x 200" in mega["sample"] and "301 solves" in mega["sample"]


def test_whole_job_alu_fraction():
    sys.path.insert(0, ROOT)
    import bench
    r = bench.whole_job_alu(2_000_000_000, 0.5, "mixed")
    assert abs(r["achieved_TFLOPs"] - 18 * 4e9 / 1e12) < 1e-12
    assert r["peak_TFLOPs"] == 78.6 and abs(r["frac"] - r["achieved_TFLOPs"] / 78.6) < 1e-15
