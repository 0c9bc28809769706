"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle_tvspec.so.

Plain gcc, no fused multiply-add, OpenMP only over independent per-pixel rows.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tvspec_oracle.c")
LIB = os.path.join(HERE, "liboracle_tvspec.so")
# the same oracle built with the address and undefined-behaviour sanitizers
# (loaded instead of LIB when TVSPEC_ORACLE_SANITIZE=1; the process then needs
# the ASan runtime preloaded, see tests/test_host_sanitized.py)
LIB_SAN = os.path.join(HERE, "liboracle_tvspec_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SAN if sanitize else LIB
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra"]
    if sanitize:
        cmd += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    cmd += ["-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
