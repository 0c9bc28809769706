"""Host code under the address and undefined-behaviour sanitizers (CPU only).

- The library's GPU-free host logic (argument validation, the band of every
  sample, the server's pool allocator; paper_2006_10004_amd/csrc/
  host_logic.cpp) is built with g++ -fsanitize=address,undefined together
  with tests/host_logic_check.cpp, which drives it over edge values and
  random sequences against a shadow model, and run.
- The FP64 oracle is built with the same sanitizers and the whole CPU test
  suite is run against it in a child process with the ASan runtime
  preloaded (leak detection off: the interpreter itself is not
  instrumented); the child checks first that the sanitized oracle is the
  library it loaded.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_host_logic_under_sanitizers(tmp_path):
    exe = tmp_path / "host_logic_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2006_10004_amd", "csrc"), "-o", str(exe),
           os.path.join(ROOT, "tests", "host_logic_check.cpp"),
           os.path.join(ROOT, "paper_2006_10004_amd", "csrc", "host_logic.cpp")]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "host logic ok" in r.stdout


@pytest.mark.slow
@pytest.mark.sanitized
def test_cpu_suite_with_sanitized_oracle():
    asan = _asan_runtime()
    if asan is None:
        pytest.skip("no ASan runtime for gcc on this host")
    sys.path.insert(0, ROOT)
    from oracle import build as oracle_build
    oracle_build.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0", TVSPEC_ORACLE_SANITIZE="1",
               PYTHONPATH=ROOT)
    probe = ("import oracle, numpy as np; r = oracle.decompose(np.random.default_rng(1).random((1, 9, 11))"
             ".astype(np.float32), 0.01, 3, 7, [0, 1, 3]); "
             "maps = open('/proc/self/maps').read(); assert 'liboracle_tvspec_san.so' in maps, 'not loaded'; "
             "print('sanitized oracle loaded')")
    p = subprocess.run([sys.executable, "-c", probe], capture_output=True, text=True, env=env, cwd=ROOT,
                       timeout=300)
    assert p.returncode == 0 and "sanitized oracle loaded" in p.stdout, p.stderr[-3000:]
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-x",
                        "-p", "no:cacheprovider", "-m", "not gpu and not sanitized"],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=1500)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "passed" in r.stdout
