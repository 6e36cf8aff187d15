#!/bin/sh
# Builds the CPU oracle (test infrastructure) as a shared library next to this
# script.  Plain C, FP64, OpenMP; -ffp-contract=off keeps every product and sum
# rounded separately, as written.
set -e
here="$(cd "$(dirname "$0")" && pwd)"
gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared -Wall -Wextra \
    -o "$here/libss_oracle.so" "$here/ss_oracle.c" -lm
