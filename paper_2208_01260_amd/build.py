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


def source_hash(csrc: str = os.path.join(HERE, "csrc"), defines=()) -> str:
    """sha256 (16 hex digits) of the solver's HIP sources, the C header and the compile flags:
    the stamp built into libswe_hweno.so and checked by the binding at load."""
    import hashlib

    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(csrc) if f.endswith((".hip", ".hpp", ".inc")) and f != "calib.hip")
    for f in files:
        h.update(f.encode() + b"\0")
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "include", "swe_hweno.h"), "rb") as fh:
        h.update(fh.read())
    h.update(" ".join(FLAGS[:-1] + sorted(defines)).encode())
    return h.hexdigest()[:16]


def build(verbose: bool = False, out: str = OUT, defines=(), src: str = SRC) -> str:
    defines = tuple(defines)
    if src != CALIB_SRC:
        defines = defines + ('SWE_HWENO_SOURCE_HASH="%s"' % source_hash(os.path.dirname(src), defines),)
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
