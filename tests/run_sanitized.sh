#!/bin/bash
# CPU test suite (-m "not gpu") with the host code under AddressSanitizer and
# UndefinedBehaviorSanitizer:
#   1. the oracle (gcc, -fsanitize=address,undefined) under every CPU test,
#      with gcc's ASan runtime preloaded into python;
#   2. the C ABI's host code (hipcc -Xarch_host -fsanitize=...) under the ABI
#      tests, with clang's ASan runtime preloaded.
# Any sanitizer report aborts the run (exit status != 0).
#     bash tests/run_sanitized.sh
set -euo pipefail
cd "$(dirname "$0")/.."
export RAYGS_SANITIZE=1
export ASAN_OPTIONS=detect_leaks=0:abort_on_error=1:verify_asan_link_order=0
export UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1
python -c "import oracle; oracle.build_library(force=True)"
echo "== oracle under gcc ASan/UBSan: python -m pytest tests -m 'not gpu' (ABI tests use the plain library)"
LD_PRELOAD="$(gcc -print-file-name=libasan.so):$(gcc -print-file-name=libubsan.so)" \
    python -m pytest tests -q -m "not gpu" -p no:cacheprovider
python -m paper_2503_18682_amd.build
RT="$(ls /opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so | head -1)"
echo "== C ABI host code under clang ASan/UBSan: python -m pytest tests/test_abi.py"
RAYGS_LIBRARY="$PWD/paper_2503_18682_amd/libraygs_san.so" LD_PRELOAD="$RT" \
    python -m pytest tests/test_abi.py -q -m "not gpu" -p no:cacheprovider
echo "sanitized CPU suite: clean"
