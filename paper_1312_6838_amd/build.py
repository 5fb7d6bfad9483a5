"""Build the gfx950 HIP library libgcss.so in-tree (hipcc, no GPU needed).

    python -m paper_1312_6838_amd.build
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgcss.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


# host code under AddressSanitizer and UndefinedBehaviorSanitizer (device
# code unchanged); the runtime is clang's shared one, preloaded by the caller
SANITIZE_FLAGS = [
    "-O1", "-g", "-fno-omit-frame-pointer",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
]


def asan_runtime() -> str:
    """Path of clang's shared AddressSanitizer runtime in the ROCm toolchain."""
    found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return sorted(found)[-1] if found else ""


def build(jobs: int | None = None, verbose: bool = False, out_dir: str | None = None,
          sanitize: bool = False) -> str:
    """Compile every source and link libgcss.so (into out_dir, default the
    package; sanitize: host code under ASan + UBSan); returns the library path."""
    bdir = os.path.join(out_dir, "_build") if out_dir else BUILD
    lib_path = os.path.join(out_dir, "libgcss.so") if out_dir else LIB
    flags = [f for f in FLAGS if f != "-O3"] + SANITIZE_FLAGS if sanitize else FLAGS
    os.makedirs(bdir, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    objs = []
    procs = []
    for src in sources():
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC, *flags, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = lib_path + ".tmp"
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-o", tmp, *objs]
    if sanitize:
        link[3:3] = ["-shared-libasan", "-Xarch_host", "-fsanitize=address,undefined"]
    if verbose:
        print(" ".join(link), flush=True)
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode())
    os.replace(tmp, lib_path)
    return lib_path


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    if p.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{out.decode()}")
    text = out.decode().strip()
    if text:
        # hipcc's host pass does not know the packed-fp32 feature; keep the rest
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
        if lines:
            print("\n".join(lines), file=sys.stderr)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
