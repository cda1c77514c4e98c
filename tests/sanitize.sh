#!/bin/bash
# CPU test suite under AddressSanitizer + UndefinedBehaviorSanitizer: the
# GPU library's host code (validation, planning, workspace sizing, the
# tuning-file parser, host-only contexts) and the FP64 oracle, both built
# with clang's sanitizers and run in one Python process with the clang
# runtime preloaded.  No GPU is used (the GPU tests are deselected).
#   bash tests/sanitize.sh [extra pytest args]
set -euo pipefail
ROOT="$(cd "$(dirname "$0")/.." && pwd)"
cd "$ROOT"
python paper_2211_08506_amd/build.py --sanitize > /dev/null
python oracle/build.py --sanitize > /dev/null
RT="$(ls /opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so | head -n 1)"
export PARTICLEGRID_LIB="$ROOT/_build/sanitize/libparticlegrid.so"
export PGORACLE_LIB="$ROOT/_build/sanitize/libpgoracle.so"
# Python itself is not instrumented: leaks of the interpreter are not ours
export ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1"
export UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1"
LD_PRELOAD="$RT" python -m pytest tests -q -m "not gpu" -p no:cacheprovider "$@"
