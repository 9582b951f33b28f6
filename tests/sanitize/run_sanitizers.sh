#!/bin/bash
# Host-code sanitizer runs of the library (CPU only): the host C++ of the
# library (engine, MPO builder) and the driver are built with
# AddressSanitizer + UndefinedBehaviorSanitizer, then with ThreadSanitizer;
# the device code is built as usual; tests/sanitize/host_driver.cpp runs the
# host-only entry points.  Usage: tests/sanitize/run_sanitizers.sh [outdir]
set -eo pipefail
ROOT=$(cd "$(dirname "$0")/../.." && pwd)
OUT=${1:-${TMPDIR:-/tmp}/tnqe_sanitize}
mkdir -p "$OUT"
HIPCC=/opt/rocm/bin/hipcc
CLANG=/opt/rocm/llvm/bin/clang++
CSRC=$ROOT/paper_2404_10223_amd/csrc
FLAGS="--offload-arch=gfx950 -g -fPIC -std=c++17 -pthread -Xclang -target-feature -Xclang -packed-fp32-ops -Wno-unused-command-line-argument -I$ROOT/include"
for f in kernels_gate kernels_svd kernels_env kernels_gep kernels_sweep noalloc; do
  [ -f "$OUT/$f.o" ] || $HIPCC $FLAGS -O3 -c "$CSRC/$f.hip" -o "$OUT/$f.o"
done
run() {   # tag, sanitizer list, runtime options variable
  local tag=$1 san=$2
  for f in engine mpo; do
    $HIPCC $FLAGS -O1 -fno-omit-frame-pointer -Xarch_host -fsanitize=$san -c "$CSRC/$f.cpp" -o "$OUT/$f.$tag.o"
  done
  $HIPCC $FLAGS -O1 -Xarch_host -fsanitize=$san -c "$ROOT/tests/sanitize/host_driver.cpp" -o "$OUT/driver.$tag.o"
  $CLANG -fsanitize=$san --hip-link --offload-arch=gfx950 -pthread -o "$OUT/driver.$tag" "$OUT/driver.$tag.o" \
    "$OUT/engine.$tag.o" "$OUT/mpo.$tag.o" "$OUT"/kernels_*.o "$OUT/noalloc.o" -L/opt/rocm/lib -lamdhip64 \
    -Wl,-rpath,/opt/rocm/lib
  echo "== $tag"
  "$OUT/driver.$tag"
}
UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 ASAN_OPTIONS=detect_leaks=1 run asan address,undefined
TSAN_OPTIONS=halt_on_error=1 run tsan thread
