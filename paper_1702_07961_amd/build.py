"""Build step of libmms: compiles the HIP sources for gfx950 with hipcc.

``python -m paper_1702_07961_amd.build`` (or ``build()``) writes
``paper_1702_07961_amd/libmms.so``.  It always recompiles.
``build(sanitize="address")`` / ``build(sanitize="thread")`` write host-side
sanitizer builds under ``_build/`` for the CPU tests of the runtime.
"""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmms.so")

SOURCES = ["mms_kernels.hip", "mms_merge_keys.hip", "mms_merge_pairs.hip", "mms_merge_heap.hip", "mms_kernels64.hip", "mms_mergepath.hip", "mms_noalloc.hip", "mms_api.cpp", "mms_server.cpp"]
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall",
    f"--offload-arch={ARCH}",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def sanitizer_runtime(kind: str) -> str:
    """The compiler's shared sanitizer runtime for `kind` ("address" or
    "thread"), to preload into an uninstrumented interpreter."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    short = {"address": "asan", "thread": "tsan"}[kind]
    found = sorted(glob.glob(os.path.join(rocm, "llvm", "lib", "clang", "*", "lib", "linux",
                                          f"libclang_rt.{short}-x86_64.so")))
    if not found:
        raise RuntimeError(f"no {short} runtime under {rocm}/llvm")
    return found[-1]


def _sources_hash() -> str:
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)) + ["../../include/mms.h"]:
        path = os.path.normpath(os.path.join(CSRC, name))
        if os.path.isfile(path):
            with open(path, "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False, jobs: int = 4, sanitize: str | None = None) -> str:
    """Compile libmms.  With sanitize = "address" or "thread" the host code
    (runtime, C ABI, serving loop) is instrumented with that sanitizer (the
    device code never is) and the library goes to _build/san_<kind>/, rebuilt
    only when a source changed; load it with MMS_LIBRARY=<path> and the
    runtime of sanitizer_runtime() preloaded."""
    out_dir = BUILD if sanitize is None else os.path.join(BUILD, f"san_{sanitize}")
    lib_path = LIB if sanitize is None else os.path.join(out_dir, f"libmms_{sanitize}.so")
    os.makedirs(out_dir, exist_ok=True)
    extra = []
    if sanitize is not None:
        if sanitize not in ("address", "thread"):
            raise ValueError(f"unknown sanitizer {sanitize!r}")
        stamp = os.path.join(out_dir, "sources.hash")
        if os.path.exists(lib_path) and os.path.exists(stamp) and open(stamp).read() == _sources_hash():
            return lib_path
        # host-side instrumentation only: each sanitizer flag behind -Xarch_host
        extra = ["-O1", "-g", "-Xarch_host", f"-fsanitize={sanitize}", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + extra
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature; that warning is expected
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed.append(src)
            print(text, file=sys.stderr)
        elif lines and verbose:
            print("\n".join(lines))
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = lib_path + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if sanitize is not None:
        cmd += ["-Xarch_host", f"-fsanitize={sanitize}", "-shared-libsan"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib_path)
    if sanitize is not None:
        with open(os.path.join(out_dir, "sources.hash"), "w") as f:
            f.write(_sources_hash())
    return lib_path


if __name__ == "__main__":
    print(build(verbose=True))
