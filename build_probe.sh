#!/bin/bash
set -e
cd "$(dirname "$0")"
mkdir -p obj
F="--offload-arch=gfx950 -O3 -std=c++17 -fPIC -Xclang -target-feature -Xclang -packed-fp32-ops -fhip-fp32-correctly-rounded-divide-sqrt"
for f in csrc/*.hip; do /opt/rocm/bin/hipcc $F -c $f -o obj/$(basename $f).o & done; wait
/opt/rocm/bin/hipcc --offload-arch=gfx950 -shared -o libgcss_probe.so obj/*.o
