#!/bin/bash
# Runs the host-model tests (the heap and round-loop logic of the GPU kernels,
# instantiated with a one-thread team on the CPU) under AddressSanitizer and
# UndefinedBehaviorSanitizer.  The sanitized library is built with the
# sanitizers on its host code only; Python itself is not instrumented, so the
# ASan runtime has to be loaded first, through LD_PRELOAD.
#
#     bash tests/hostmodel/asan.sh [pytest arguments]
set -e
HERE="$(cd "$(dirname "${BASH_SOURCE[0]}")" && pwd)"
RT="$(/opt/rocm/llvm/bin/clang -print-file-name=libclang_rt.asan-x86_64.so)"
if [ ! -f "$RT" ]; then
  echo "ASan runtime not found ($RT)" >&2
  exit 2
fi
cd "$HERE/../.."
PBH_HOSTMODEL_ASAN=1 LD_PRELOAD="$RT" ASAN_OPTIONS=detect_leaks=0 \
  python -m pytest tests/test_hostmodel.py -q -p no:cacheprovider "$@"
