#!/bin/sh
# Builds the FP64 oracle (test infrastructure) as oracle/liborc.so.
set -e
cd "$(dirname "$0")"
gcc -O2 -std=c11 -D_GNU_SOURCE -fopenmp -fPIC -shared -ffp-contract=off -fno-fast-math -Wall -Wextra \
    orc.c -o liborc.so -lm
