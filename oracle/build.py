"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so with g++.

With sanitize=True the build goes to oracle/liboracle_san.so, instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer (every finding aborts); oracle.py loads it
when the environment variable GPSS_SANITIZED is "oracle", in a process that preloads g++'s
libasan and libubsan (tests/run_sanitized.sh)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
LIB_SAN = os.path.join(HERE, "liboracle_san.so")
SOURCES = [os.path.join(HERE, "oracle.cpp")]
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    lib = LIB_SAN if sanitize else LIB
    cmd = ["g++", "-std=c++17", "-O1" if sanitize else "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-Wno-unused-parameter", *(SANITIZE if sanitize else []), "-o", lib + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)
