#!/bin/sh
# Builds the C oracle (FP64, OpenMP) next to this script: oracle/liboracle.so
set -e
cd "$(dirname "$0")"
gcc -O2 -std=c99 -fopenmp -fPIC -shared -Wall -Wextra -o liboracle.so.tmp hisq_oracle.c
mv liboracle.so.tmp liboracle.so
