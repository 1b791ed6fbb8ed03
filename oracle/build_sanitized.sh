#!/bin/sh
# Builds the CPU oracle with AddressSanitizer and UndefinedBehaviorSanitizer as
# $1/liboracle_asan.so (default: oracle/), for running the oracle's tests under
# the sanitizers (load it through SQA_ORACLE_LIB with gcc's libasan and libubsan
# preloaded).  Same sources and floating-point flags as build.sh.
set -e
cd "$(dirname "$0")"
out="${1:-.}"
gcc -std=gnu99 -O1 -g -fno-omit-frame-pointer -fsanitize=address,undefined -fno-sanitize-recover=undefined \
    -fno-fast-math -ffp-contract=off -fPIC -shared -Wall -Wextra \
    -o "$out/liboracle_asan.so" philox.c embed.c tables.c sqa.c wolff.c pt.c decode.c -lm -lpthread
