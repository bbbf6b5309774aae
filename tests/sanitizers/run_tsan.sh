#!/bin/bash
# Builds the library's host code and the server driver with a host sanitizer
# (SAN=thread, the default, or SAN=address for AddressSanitizer with
# UndefinedBehaviorSanitizer; device code as usual) into a scratch folder and
# runs the driver on the GPU.
set -e
ROOT=$(cd "$(dirname "$0")/../.." && pwd)
OUT=${TSAN_OUT:-$(mktemp -d)}
HIPCC=${HIPCC:-/opt/rocm/bin/hipcc}
FLAGS="--offload-arch=gfx950 -O1 -g -std=c++17 -fPIC -Xclang -target-feature -Xclang -packed-fp32-ops -ffp-contract=fast -I $ROOT/include"
SAN=${SAN:-thread}
if [ "$SAN" = thread ]; then HOSTSAN="-Xarch_host -fsanitize=thread"; else HOSTSAN="-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined"; fi
OBJS=""
for f in dmx_lib kern_free_small kern_free kern_free_wide kern_tree kern_stack; do
  if [ "$f" = dmx_lib ]; then SANF="$HOSTSAN"; else SANF=""; fi
  $HIPCC $FLAGS $SANF -c -o "$OUT/$f.o" "$ROOT/paper_2506_14186_amd/csrc/$f.hip" &
  OBJS="$OBJS $OUT/$f.o"
done
wait
$HIPCC $FLAGS $HOSTSAN -c -o "$OUT/server_$SAN.o" "$ROOT/tests/sanitizers/server_tsan.cpp"
$HIPCC --offload-arch=gfx950 $HOSTSAN -o "$OUT/server_$SAN" "$OUT/server_$SAN.o" $OBJS
echo "built $OUT/server_$SAN"
if [ "${TSAN_BUILD_ONLY:-0}" = 1 ]; then exit 0; fi
TSAN_OPTIONS="halt_on_error=0 second_deadlock_stack=1" ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0" \
  UBSAN_OPTIONS="print_stacktrace=1" "$OUT/server_$SAN"
