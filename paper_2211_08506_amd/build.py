"""Build the gfx950 HIP library libparticlegrid.so in-tree.

    python paper_2211_08506_amd/build.py        (or __graft_entry__.build())

(Run as a file: importing it through the package would first load the
library it is about to rebuild.)

Every translation unit is compiled with hipcc for gfx950 only, with FP
contraction off (the exact window predicate relies on error-free
transforms evaluated as written; fused multiply-adds are spelled out where
wanted) and packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libparticlegrid.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["pg_api.cpp", "pg_window.hip", "pg_plain.hip", "pg_adjoint.hip", "pg_crystal.hip",
           "pg_reversal.hip", "pg_triclinic.hip", "pg_scratch.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # MFMA accumulators in ordinary VGPRs (gfx950 reads and writes them
          # there): no copies to and from AGPRs around every MFMA
          "-mllvm", "-amdgpu-mfma-vgpr-form=1",
          "-Wall", "-Wno-unused-result", "-Wno-unused-value", "-I", os.path.join(ROOT, "include")]


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer (the runtime's
# validation, planning, workspace sizing and tuning-file parser; the device
# code is built as usual).  For CPU-only test runs: the library then needs
# the clang sanitizer runtime preloaded, as tests/sanitize.sh does.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all",
            "-Xarch_host", "-shared-libsan"]


def _compile(src: str, verbose: bool, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + COMMON + list(extra) + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Build the library in-tree, or with sanitize=True a host-sanitized copy
    at _build/sanitize/libparticlegrid.so (the in-tree library is left as it
    is)."""
    bdir = os.path.join(BUILD, "sanitize") if sanitize else BUILD
    lib = os.path.join(bdir, "libparticlegrid.so") if sanitize else LIB
    extra = SANITIZE if sanitize else []
    os.makedirs(bdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, bdir, extra), SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + list(extra) + objs + \
        ["-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, sanitize="--sanitize" in sys.argv[1:]))
