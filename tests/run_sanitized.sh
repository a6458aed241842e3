#!/bin/bash
# The CPU test suite (-m "not gpu") against sanitized host builds, in two passes:
#   1. the oracle built by g++ with AddressSanitizer and UndefinedBehaviorSanitizer
#      (oracle/liboracle_san.so, selected by GPSS_SANITIZED=oracle);
#   2. the library's host code (C ABI, argument validation, scene set-up) built by clang with
#      the same two sanitizers (paper_2603_00280_amd/libgpss_san.so, GPSS_SANITIZED=abi).
# The g++ and clang sanitizer runtimes cannot share a process, hence two passes, each
# preloading its runtime into the Python interpreter.  Every finding aborts the run.
# Usage: tests/run_sanitized.sh [extra pytest arguments]
set -euo pipefail
ROOT=$(cd "$(dirname "$0")/.." && pwd)
cd "$ROOT"
python3 -m oracle.build --sanitize
python3 -m paper_2603_00280_amd.build --sanitize
# leaks: the interpreter and its extension modules hold memory until exit by design
export ASAN_OPTIONS=detect_leaks=0:abort_on_error=1
export UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1
GCC_RT="$(g++ -print-file-name=libasan.so):$(g++ -print-file-name=libubsan.so)"
CLANG_RT="$(/opt/rocm/llvm/bin/clang -print-resource-dir)/lib/linux/libclang_rt.asan-x86_64.so"
echo "== pass 1: oracle under g++ ASan + UBSan"
GPSS_SANITIZED=oracle LD_PRELOAD="$GCC_RT" python3 -m pytest tests/ -q -m "not gpu" -p no:cacheprovider "$@"
echo "== pass 2: C ABI under clang ASan + UBSan"
GPSS_SANITIZED=abi LD_PRELOAD="$CLANG_RT" python3 -m pytest tests/ -q -m "not gpu" -p no:cacheprovider "$@"
