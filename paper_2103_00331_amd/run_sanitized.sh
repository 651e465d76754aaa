#!/bin/bash
# Host-side AddressSanitizer / UndefinedBehaviorSanitizer run: build the
# sanitizer variant of the library (host code instrumented, device code as
# usual) and run the CPU tests against it -- the ABI checks (create,
# validation, classification, layouts, Tucker -> Tensor-Train rewrite, batch
# and MLP argument checks) and the oracle pins.  No GPU is used.
set -euo pipefail
HERE=$(cd "$(dirname "$0")" && pwd)
ROOT=$(dirname "$HERE")
cd "$ROOT"
python3 "$HERE/build.py" --sanitize
RT=$(/opt/rocm/llvm/bin/clang -print-file-name=libclang_rt.asan-x86_64.so)
export CPMDP_LIBRARY="$HERE/libcpmdp_san.so"
export ASAN_OPTIONS=detect_leaks=0:verify_asan_link_order=0:abort_on_error=1
export UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1
LD_PRELOAD="$RT" python3 -m pytest tests -q -m "not gpu" -p no:cacheprovider "$@"
