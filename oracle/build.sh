#!/bin/sh
# Builds the CPU oracle (test infrastructure) as oracle/liboracle.so.
# Plain C, no fast-math, no floating-point contraction, host libm.
set -e
cd "$(dirname "$0")"
gcc -std=gnu99 -O2 -fno-fast-math -ffp-contract=off -fPIC -shared -Wall -Wextra \
    -o liboracle.so philox.c embed.c tables.c sqa.c wolff.c pt.c decode.c -lm -lpthread
