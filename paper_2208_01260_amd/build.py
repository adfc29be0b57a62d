"""Build libswe_hweno.so in-tree with hipcc for gfx950 (no JIT cache, no site-packages)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "swe_hweno.hip")
OUT = os.path.join(HERE, "libswe_hweno.so")
CALIB_SRC = os.path.join(HERE, "csrc", "calib.hip")
CALIB_OUT = os.path.join(HERE, "libswe_hweno_calib.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, out: str = OUT, defines=(), src: str = SRC) -> str:
    cmd = [HIPCC] + FLAGS + ["-D" + d for d in defines] + [src, "-o", out + ".tmp"]
    if verbose:
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + src)
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(out + ".tmp", out)
    return out


def build_calib(verbose: bool = False) -> str:
    """The device calibration library (sustained FP64 FMA stream) used by bench.py."""
    return build(verbose, out=CALIB_OUT, src=CALIB_SRC)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    print(build_calib(verbose="-v" in sys.argv))
