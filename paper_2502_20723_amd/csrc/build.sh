#!/bin/bash
# Build libtdo.so for gfx950 (MI355X).  Usage: build.sh [out_dir]
set -euo pipefail
here="$(cd "$(dirname "$0")" && pwd)"
out="${1:-$here/..}"
mkdir -p "$here/_build"
srcs=(api lindblad net_pack net_fwd net_bwd net_bwd_mlp net_bwd_attn train sampler batched observables optim sr noalloc jvp)
objs=()
pids=()
for s in "${srcs[@]}"; do
  obj="$here/_build/$s.o"
  objs+=("$obj")
  /opt/rocm/bin/hipcc --offload-arch=gfx950 -O3 -std=c++17 -fPIC -Wall -Wno-unused-result \
    -Xclang -target-feature -Xclang -packed-fp32-ops -munsafe-fp-atomics \
    -c "$here/$s.hip" -o "$obj" 2> "$here/_build/$s.log" &
  pids+=($!)
done
rc=0
for i in "${!pids[@]}"; do
  if ! wait "${pids[$i]}"; then
    echo "compile failed: ${srcs[$i]}.hip" >&2
    grep -v "packed-fp32-ops" "$here/_build/${srcs[$i]}.log" >&2 || true
    rc=1
  fi
done
[ $rc -eq 0 ] || exit $rc
/opt/rocm/bin/hipcc --offload-arch=gfx950 -shared -fPIC "${objs[@]}" -o "$out/libtdo.so.tmp"
mv "$out/libtdo.so.tmp" "$out/libtdo.so"
echo "built $out/libtdo.so"
