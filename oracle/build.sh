#!/bin/sh
# Builds the FP64 CPU reference (test infrastructure) as liboracle.so.
# It compiles its own copy of the seeded primitive generator.
#   sh build.sh            -> liboracle.so
#   sh build.sh sanitize   -> liboracle_san.so, with AddressSanitizer and
#                             UndefinedBehaviorSanitizer (any finding aborts);
#                             load it with libasan preloaded
set -e
here="$(cd "$(dirname "$0")" && pwd)"
out="$here/liboracle.so"
extra=""
if [ "$1" = "sanitize" ]; then
    out="$here/liboracle_san.so"
    extra="-g -fno-omit-frame-pointer -fsanitize=address,undefined -fno-sanitize-recover=all"
fi
gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -fopenmp -Wall -Wextra -Wno-unused-parameter $extra \
    -I"$here/../paper_2110_13055_amd/inputs" \
    "$here/cdi_oracle.c" "$here/../paper_2110_13055_amd/inputs/geomgen.c" \
    -lm -o "$out"
