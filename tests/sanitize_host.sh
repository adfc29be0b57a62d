#!/usr/bin/env bash
# Host-side sanitizer run, CPU only (no GPU needed or used).
#   1. The oracle built by g++ with AddressSanitizer and UndefinedBehaviorSanitizer (single
#      threaded: no OpenMP) runs its pins: the oracle's building blocks, scheme and tangent tests
#      (the "slow" ones excepted).
#   2. The solver library's host code (argument validation, context set-up, the C ABI) built by
#      hipcc with clang's AddressSanitizer and UBSan on the host side only (-Xarch_host; the
#      device code is not instrumented) runs the ABI tests, which exercise every entry point's
#      host-side validation without touching a device.
# Works in a temporary copy of the repository, so the tree's own builds are left alone. Exits
# non-zero on any sanitizer report or test failure.
set -euo pipefail
ROOT=$(cd "$(dirname "$0")/.." && pwd)
TMP=$(mktemp -d)
trap 'rm -rf "$TMP"' EXIT
(cd "$ROOT" && tar cf - --exclude=.git --exclude=_work --exclude=gpurun_out --exclude='*.so' .) | (cd "$TMP" && tar xf -)
cd "$TMP"

echo "== oracle: g++ -fsanitize=address,undefined"
make -s -C oracle liboracle.so \
  CXXFLAGS="-std=c++17 -O1 -g -ffp-contract=off -fPIC -fno-omit-frame-pointer -fsanitize=address,undefined -fno-sanitize-recover=undefined -Wall -Wextra -Wno-unused-parameter -Wno-unknown-pragmas"
GASAN="$(gcc -print-file-name=libasan.so) $(gcc -print-file-name=libubsan.so)"
ASAN_OPTIONS=detect_leaks=0:abort_on_error=1 UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1 \
  LD_PRELOAD="$GASAN" ORACLE_THREADS=1 \
  python -m pytest tests/test_oracle_blocks.py tests/test_oracle_scheme.py tests/test_oracle_tangents.py \
  -m "not slow and not gpu" -q -p no:cacheprovider

echo "== solver library host code: hipcc -Xarch_host -fsanitize=address,undefined"
STAMP=$(python -c "from paper_2208_01260_amd.build import source_hash; print(source_hash())")
/opt/rocm/bin/hipcc --offload-arch=gfx950 -O1 -g -std=c++17 -fPIC -shared \
  -Xclang -target-feature -Xclang -packed-fp32-ops \
  -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer \
  -Xarch_host -fno-sanitize-recover=undefined \
  -Iinclude "-DSWE_HWENO_SOURCE_HASH=\"$STAMP\"" \
  paper_2208_01260_amd/csrc/swe_hweno.hip -o paper_2208_01260_amd/libswe_hweno.so 2> build_asan.log || {
  cat build_asan.log; exit 1; }
python -c "from paper_2208_01260_amd import build; build.build_calib()"
CASAN=$(ls /opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so | head -1)
ASAN_OPTIONS=detect_leaks=0:abort_on_error=1 UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1 \
  LD_PRELOAD="$CASAN" python -m pytest tests/test_abi.py -q -p no:cacheprovider
echo "== sanitizers: clean"
