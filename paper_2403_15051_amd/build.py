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
# Sanitized build of the host code only (AddressSanitizer + UndefinedBehaviorSanitizer): the host-code
# sources (HOST_SOURCES: tables, ABI) are compiled with every sanitizer flag reaching the host
# compilation alone; the kernel sources (device code and their launch wrappers) link as the ordinary
# build's objects, compiled first when missing or older than their sources and headers.  The
# result (SAN_LIB) needs clang's ASan runtime preloaded into the process (san_runtime()); it is
# for the CPU tests of the host tables, selected with LBE_LIB=SAN_LIB.
HOST_SOURCES = ["lbe_tables.cpp", "lbe_abi.cpp"]
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


def _fresh(obj: str, deps) -> bool:
    return os.path.exists(obj) and all(os.path.getmtime(obj) >= os.path.getmtime(d) for d in deps)


def build(verbose: bool = False, sanitize: bool = False) -> str:
    objdir = os.path.join(OBJ, "san") if sanitize else OBJ
    lib = SAN_LIB if sanitize else LIB
    os.makedirs(objdir, exist_ok=True)
    os.makedirs(OBJ, exist_ok=True)
    headers = [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    headers.append(os.path.join(os.path.dirname(HERE), "include", "lbe.h"))
    jobs, objs = [], []  # (source, extra flags, object folder) to compile; objects ready to link
    for name in SOURCES:
        src = os.path.join(CSRC, name)
        if not sanitize:
            jobs.append((src, [], OBJ))
        elif name in HOST_SOURCES:
            jobs.append((src, SAN_FLAGS, objdir))
        elif _fresh(os.path.join(OBJ, os.path.splitext(name)[0] + ".o"), [src] + headers):
            objs.append(os.path.join(OBJ, os.path.splitext(name)[0] + ".o"))
        else:
            jobs.append((src, [], OBJ))
    with cf.ThreadPoolExecutor(max_workers=max(1, len(jobs))) as ex:
        objs += list(ex.map(lambda j: _compile(j[0], verbose, j[1], j[2]), jobs))
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
