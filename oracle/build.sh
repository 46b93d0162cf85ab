#!/bin/sh
# Builds the CPU oracle (test infrastructure only) as a shared library next to this script.
set -e
cd "$(dirname "$0")"
gcc -O2 -fPIC -shared -std=c99 -Wall -Wextra -Wno-unused-parameter -fno-fast-math \
    -ffp-contract=off -fopenmp -o libccz4_oracle.so ccz4_rhs_point.c ccz4_oracle.c ccz4_mlp.c -lm
