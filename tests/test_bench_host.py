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
    other = tmp_path / "engine.hip"
    other.write_text(open(bench.KERNEL_SOURCE).read() + "\n// edited\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(other))
    assert bench.measured_traffic("mixed", 0) is None
