"""Build libdg.so (HIP kernels for gfx950 + the C-ABI) in-tree with hipcc.

The kernel source is compiled once per part (DG_PART = 0..5: stage kernels
of order 1 with the set-up kernels, limiter, network, batched launches, stage
kernels of orders 2 and 3) and the C++ sources once each, all in
parallel, then linked into one shared library."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdg.so")
KERNEL_SOURCE = "dg_kernels.hip"
KERNEL_PARTS = 6
SOURCES = ["dg_tables.cpp", "dg_api.cpp", "dg_batch.cpp"]
ARCH = os.environ.get("DG_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for all device code (some of their
# forms are not trusted on this target); FP64 arithmetic is unaffected.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=on"]


def _jobs():
    units = [(KERNEL_SOURCE, part, f"dg_kernels_part{part}.o") for part in range(KERNEL_PARTS)]
    units += [(src, None, src + ".o") for src in SOURCES]
    return units


def build(verbose=False):
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    procs, objs = [], []
    for src, part, oname in _jobs():
        obj = os.path.join(build_dir, oname)
        cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
               "-Wno-unused-function", "-I", os.path.join(HERE, "..", "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        if part is not None:
            cmd[1:1] = DEVICE_FLAGS + [f"-DDG_PART={part}"]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [cmd for cmd, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
