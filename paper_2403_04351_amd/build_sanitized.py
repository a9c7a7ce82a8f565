"""Builds a host-sanitized copy of the ltd library (AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only; the device code is built
normally) under _build/sanitize/, for running the host-side ABI tests on a
machine without a GPU.  Load it with LTD_LIBRARY=<path> and the ASan runtime
preloaded (``asan_runtime()``)."""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

from . import build as b

OUT = os.path.join(b.BUILD, "sanitize")
LIB = os.path.join(OUT, "libltd.so")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def clang_dir() -> str:
    cands = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux"))
    if not cands:
        raise RuntimeError("clang runtime directory not found")
    return cands[-1]


def asan_runtime() -> str:
    p = os.path.join(clang_dir(), "libclang_rt.asan-x86_64.so")
    if not os.path.exists(p):
        raise RuntimeError(f"{p} not found")
    return p


def _compile(src: str) -> str:
    obj = os.path.join(OUT, os.path.splitext(src)[0] + ".o")
    flags = [f if f != "-O3" else "-O1" for f in b.FLAGS] + ["-g"]
    cmd = [b.hipcc(), *flags, *b.EXTRA.get(src, []), *HOST_SAN, "-c", os.path.join(b.CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(b.SOURCES)) as ex:
        objs = list(ex.map(_compile, b.SOURCES))
    # the objects carry their device code; the shared library is a host link
    cxx = "/opt/rocm/llvm/bin/clang++"
    tmp = LIB + ".tmp"
    cmd = [cxx, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libsan", "-o", tmp, *objs,
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-Wl,-rpath," + clang_dir()]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB
