#!/bin/bash
# Host-only checks of the CPU oracle itself (test infrastructure, never the library): builds
# imin_oracle.c with gcc under AddressSanitizer + UndefinedBehaviorSanitizer and under
# ThreadSanitizer, into a temporary directory, and runs the oracle's pin tests against each
# build (IMIN_ORACLE_LIB selects the build; the sanitizer runtime is preloaded into Python).
# The threaded form of the oracle (samples split over host threads) runs under both.
# PYTHON names the interpreter (default python3).
set -euo pipefail
ROOT=$(cd "$(dirname "$0")/.." && pwd)
T=$(mktemp -d)
trap 'rm -rf "$T"' EXIT
SRC="$ROOT/oracle/imin_oracle.c"
COMMON=(-O1 -g -std=c99 -shared -fPIC -pthread -fno-omit-frame-pointer)
gcc "${COMMON[@]}" -fsanitize=address,undefined -fno-sanitize-recover=undefined \
    -o "$T/asan_ubsan.so" "$SRC" -lm
gcc "${COMMON[@]}" -fsanitize=thread -o "$T/tsan.so" "$SRC" -lm
cd "$ROOT"
PINS=(tests/test_oracle_pins.py tests/test_oracle_greedy.py tests/test_oracle_lt.py
      tests/test_oracle_counters_threads.py)
echo "[sanitize] address + undefined behaviour"
IMIN_ORACLE_LIB="$T/asan_ubsan.so" LD_PRELOAD="$(gcc -print-file-name=libasan.so)" \
    ASAN_OPTIONS=detect_leaks=0:abort_on_error=1 UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 \
    "${PYTHON:-python3}" -m pytest -q -x -s -p no:cacheprovider "${PINS[@]}"
echo "[sanitize] threads"
IMIN_ORACLE_LIB="$T/tsan.so" LD_PRELOAD="$(gcc -print-file-name=libtsan.so)" \
    TSAN_OPTIONS=halt_on_error=1 \
    "${PYTHON:-python3}" -m pytest -q -x -s -p no:cacheprovider tests/test_oracle_counters_threads.py
