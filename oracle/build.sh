#!/bin/sh
# Builds the FP64 CPU reference (test infrastructure) as liboracle.so.
# It compiles its own copy of the seeded primitive generator.
set -e
here="$(cd "$(dirname "$0")" && pwd)"
gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -fopenmp -Wall -Wextra -Wno-unused-parameter \
    -I"$here/../paper_2110_13055_amd/inputs" \
    "$here/cdi_oracle.c" "$here/../paper_2110_13055_amd/inputs/geomgen.c" \
    -lm -o "$here/liboracle.so"
