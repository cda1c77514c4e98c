"""Compile the FP64 oracle (plain C, -O2, no fast-math, no FMA contraction)
into oracle/libpgoracle.so.  Test infrastructure only."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pg_oracle.c")
LIB = os.path.join(HERE, "libpgoracle.so")


SAN_DIR = os.path.join(os.path.dirname(HERE), "_build", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang"


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """gcc -O2 in-tree; with sanitize=True an AddressSanitizer +
    UndefinedBehaviorSanitizer copy at _build/sanitize/libpgoracle.so, built
    with the clang whose sanitizer runtime the sanitized GPU library uses
    (one runtime serves both in a CPU test run)."""
    if sanitize:
        os.makedirs(SAN_DIR, exist_ok=True)
        lib = os.path.join(SAN_DIR, "libpgoracle.so")
        cmd = [CLANG, "-O1", "-g", "-std=gnu11", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", "-Wall", "-Wextra", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-shared-libsan", SRC,
               "-o", lib + ".tmp", "-lm"]
    else:
        lib = LIB
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", "-Wall", "-Wextra", SRC, "-o", lib + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
    sys.exit(0)
