"""Build liblbe.so (HIP for gfx950) in-tree with hipcc: one object per source, compiled in
parallel, then linked."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbe.so")
SOURCES = ["lbe_tables.cpp", "lbe_abi.cpp", "lbe_kernels.hip", "lbe_mlp.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-x", "hip",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-pthread",
]
# Sanitized build of the host code only (AddressSanitizer + UndefinedBehaviorSanitizer): every
# sanitizer flag reaches the host compilation alone, the device code is built as usual.  The
# result (SAN_LIB) needs clang's ASan runtime preloaded into the process (san_runtime()); it is
# for the CPU tests of the host tables, selected with LBE_LIB=SAN_LIB.
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-g"]
SAN_LINK = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-shared-libsan"]
SAN_LIB = os.path.join(OBJ, "san", "liblbe.so")


def san_runtime() -> str:
    """clang's shared ASan runtime (with the UBSan handlers) to preload for SAN_LIB."""
    import glob

    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise FileNotFoundError("clang ASan runtime not found under /opt/rocm/llvm")
    return hits[-1]


def _compile(src: str, verbose: bool, extra=(), objdir: str = OBJ) -> str:
    obj = os.path.join(objdir, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    objdir = os.path.join(OBJ, "san") if sanitize else OBJ
    lib = SAN_LIB if sanitize else LIB
    os.makedirs(objdir, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    extra = SAN_FLAGS if sanitize else []
    with cf.ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, extra, objdir), srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *(SAN_LINK if sanitize else []), "-o", tmp,
           *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
