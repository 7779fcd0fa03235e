"""Builds a copy of libsharp.so whose host code (the C ABI, plan set-up, tile
and strip lists, batch bookkeeping) is instrumented with AddressSanitizer and
UndefinedBehaviorSanitizer.  Device code is not instrumented: the kernel
objects of the regular build are linked in unchanged.  CPU use only: the
library needs the sanitizer runtime preloaded (`runtime()`), and is meant for
the host-only entry points (plan creation, validation, sizes, lists)."""
from __future__ import annotations

import glob
import os
import subprocess

from .build import BUILD, CSRC, FLAGS, HIPCC, SOURCES

HOST_SOURCES = [s for s in SOURCES if s.endswith(".cpp")]
# every sanitizer flag applies to the host pass only
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined", "-g"]


def runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (to be preloaded)."""
    llvm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    hits = sorted(glob.glob(os.path.join(llvm, "lib", "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so not found under the ROCm LLVM")
    return hits[-1]


def build(out_dir: str) -> str:
    """Compile the host sources with the sanitizers into `out_dir` and link
    them with the regular build's kernel objects (which must exist)."""
    os.makedirs(out_dir, exist_ok=True)
    kernels = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in SOURCES if s.endswith(".hip")]
    missing = [k for k in kernels if not os.path.exists(k)]
    if missing:
        raise FileNotFoundError(f"build the library first (missing {missing})")
    objs = []
    procs = []
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *[f for f in FLAGS if f != "-O3"], "-O1", *SAN, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    for cmd, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
    lib = os.path.join(out_dir, "libsharp_hostsan.so")
    # the sanitizer runtime is not linked in: it is preloaded into the process
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, *kernels, "-o", lib]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return lib
