#!/bin/sh
# Builds the CPU oracle (test infrastructure) into oracle/liboracle.so.
# No fused multiply-add: every + and * of the oracle is one rounded operation.
set -e
cd "$(dirname "$0")"
gcc -O3 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared -Wall -o liboracle.so.tmp oracle.c -lm
mv liboracle.so.tmp liboracle.so
