#!/bin/sh
# Builds the plain C oracle (test infrastructure; see adct_oracle.c).
set -e
here=$(cd "$(dirname "$0")" && pwd)
gcc -O2 -fopenmp -fPIC -shared -o "$here/libadct_oracle.so" "$here/adct_oracle.c"
