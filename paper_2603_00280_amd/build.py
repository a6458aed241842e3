"""Build libgpss.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgpss.so")
SOURCES = ["gpss_api.hip", "gpss_forward.hip", "gpss_wavefront.hip", "gpss_adjoint.hip", "gpss_batch.hip",
           "gpss_persistent.hip", "gpss_noalloc.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("GPSS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-std=c++17", "-O3", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse multiply-adds only within a source expression: the one-thread-per-path and the
    # wavefront kernels then round every shared computation identically
    "-ffp-contract=on",
    # hardware floating-point atomics for gradient accumulation (device memory from hipMalloc)
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, extra=None) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], "-c", os.path.join(CSRC, src), "-o", obj]
        if extra:
            cmd += list(extra)
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
