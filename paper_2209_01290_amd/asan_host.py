"""Build ``libpm_asan.so``: the library with its host sources (argument
validation, parameter helpers, tuning tables, job-table layout) compiled
with AddressSanitizer; the device objects are those of the normal build.
The sanitizer applies to host code only (each -fsanitize flag follows
-Xarch_host). Used by the CPU test of the host runtime.

    python -m paper_2209_01290_amd.asan_host
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

from . import build as pmbuild

PKG = pmbuild.PKG
BUILD = os.path.join(PKG, "_build_asan")
LIB = os.path.join(PKG, "libpm_asan.so")
ASAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def runtime() -> str:
    """Path of the shared AddressSanitizer runtime (for LD_PRELOAD)."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("AddressSanitizer runtime not found under /opt/rocm/llvm")
    return hits[-1]


def build(jobs: int | None = None) -> str:
    pmbuild.build(verbose=False)                 # device objects of the normal build
    os.makedirs(BUILD, exist_ok=True)
    deps = max(os.path.getmtime(d) for d in pmbuild._deps())
    hosts = sorted(glob.glob(os.path.join(pmbuild.CSRC, "*.cpp")))
    todo, objs = [], []
    for src in hosts:
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        objs.append(obj)
        if not os.path.exists(obj) or os.path.getmtime(obj) < max(os.path.getmtime(src), deps):
            todo.append((src, obj))
    with cf.ThreadPoolExecutor(jobs or min(8, os.cpu_count() or 4)) as ex:
        list(ex.map(lambda so: pmbuild._compile(so[0], so[1], ASAN_HOST + ["-g"]), todo))
    dev_objs = [os.path.join(pmbuild.BUILD, os.path.basename(s) + ".o")
                for s in sorted(glob.glob(os.path.join(pmbuild.CSRC, "*.hip")))]
    if todo or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(o) for o in objs + dev_objs):
        cmd = [pmbuild.HIPCC, "--offload-arch=" + pmbuild.ARCH, "-shared", "-fPIC", "-Xarch_host",
               "-fsanitize=address", "-shared-libsan", "-o", LIB] + objs + dev_objs
        p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if p.returncode != 0:
            raise RuntimeError("asan link failed:\n" + pmbuild._filter(p.stdout))
    return LIB


if __name__ == "__main__":
    print(build())
