"""Build libgpss.so (HIP, gfx950) in-tree with hipcc.

With sanitize=True the build goes to libgpss_san.so, its host code (the C ABI, argument
validation, scene set-up) instrumented with AddressSanitizer and UndefinedBehaviorSanitizer;
device code is built as usual.  gpss.py loads it when the environment variable GPSS_SANITIZED
is "abi", in a process that preloads clang's ASan runtime (tests/run_sanitized.sh)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgpss.so")
LIB_SAN = os.path.join(HERE, "libgpss_san.so")
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
# host code only: each sanitizer flag goes to the host compilation
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False, extra=None, sanitize: bool = False) -> str:
    lib = LIB_SAN if sanitize else LIB
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + (".san.o" if sanitize else ".o"))
        cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], "-c", os.path.join(CSRC, src), "-o", obj]
        if sanitize:
            cmd += SANITIZE
        if extra:
            cmd += list(extra)
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    # roctx: the entry points' host-side ranges
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", lib + ".tmp", *objs, "-lrocprofiler-sdk-roctx"]
    if sanitize:
        cmd += SANITIZE + ["-shared-libasan"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)
