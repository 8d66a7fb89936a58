#!/bin/bash
# Run the oracle under AddressSanitizer + UndefinedBehaviorSanitizer and under
# ThreadSanitizer, on the CPU: each instrumented build of bdf_oracle.c is
# loaded by the whole CPU test suite (BDFX_ORACLE_LIB) and by a 1,024-cell
# OpenMP batch of the mixed workload.  Any report aborts the run.
# Usage: bash oracle/sanitize.sh [workdir]
set -euo pipefail
ROOT="$(cd "$(dirname "$0")/.." && pwd)"
WORK="${1:-$(mktemp -d)}"
mkdir -p "$WORK"
SRC="$ROOT/oracle/bdf_oracle.c"
CFLAGS="-O1 -g -fno-omit-frame-pointer -std=c11 -fPIC -shared -fopenmp -ffp-contract=off"

gcc $CFLAGS -fsanitize=address,undefined -fno-sanitize-recover=all -o "$WORK/liboracle_asan.so" "$SRC" -lm
gcc $CFLAGS -fsanitize=thread -o "$WORK/liboracle_tsan.so" "$SRC" -lm

batch() {
  python3 - <<'PY'
import sys
sys.path.insert(0, sys.argv[1] if len(sys.argv) > 1 else ".")
from oracle import oracle as O
from paper_2405_01713_amd import workloads as W
w = W.make_workload("mixed_s9_s53_1m", 1024)
y, st = O.integrate(w["mechs"], w["y0"], 0.0, w["t_out"], w["rtol"], w["atol"], T=w["T"],
                    cell_mech=w["cell_mech"], nthreads=8)
assert (st["status"] == 0).all()
print("batch of", len(st), "cells on", O.max_threads(), "threads: ok")
PY
}

cd "$ROOT"
echo "== ASan + UBSan: CPU test suite"
ASAN_OPTIONS=detect_leaks=0:abort_on_error=1 UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 \
  LD_PRELOAD="$(gcc -print-file-name=libasan.so):$(gcc -print-file-name=libubsan.so)" \
  BDFX_ORACLE_LIB="$WORK/liboracle_asan.so" \
  python3 -m pytest tests -q -m "not gpu" -p no:cacheprovider -k "not pins_bite"
echo "== ASan + UBSan: 1,024-cell OpenMP batch"
ASAN_OPTIONS=detect_leaks=0:abort_on_error=1 UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 \
  LD_PRELOAD="$(gcc -print-file-name=libasan.so):$(gcc -print-file-name=libubsan.so)" \
  BDFX_ORACLE_LIB="$WORK/liboracle_asan.so" batch
echo "== TSan: 1,024-cell OpenMP batch"
TSAN_OPTIONS="halt_on_error=1 report_signal_unsafe=0 ignore_noninstrumented_modules=1" \
  LD_PRELOAD="$(gcc -print-file-name=libtsan.so)" \
  BDFX_ORACLE_LIB="$WORK/liboracle_tsan.so" batch
echo "sanitizers: clean"
