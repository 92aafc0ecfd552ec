"""Build ``libpm.so`` (HIP kernels for gfx950 plus the C-ABI host runtime).

Every ``csrc/*.hip`` and ``csrc/*.cpp`` file is compiled by hipcc in parallel
into ``_build/`` and linked into ``paper_2209_01290_amd/libpm.so``. The
``poison`` variant (``libpm_poison.so``, objects in ``_build_poison/``) is the
same library with PM_POISON_LDS=1: every LDS exchange first fills the row's
LDS with words above every modulus, a debugging build that turns a missing
barrier or an unwritten slot into a wrong result. Usage:

    python -m paper_2209_01290_amd.build [--force] [-j N] [--variant poison]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # no packed fp32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _deps():
    return glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(CSRC, "*.inc")) + \
        [os.path.join(ROOT, "include", "pm.h")]


def _filter(out: str) -> str:
    # hipcc's host pass does not know the packed-fp32 feature flag; harmless.
    return "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)


VARIANTS = {"": ([], "_build", "libpm.so"), "poison": (["-DPM_POISON_LDS=1"], "_build_poison", "libpm_poison.so")}


def _compile(src: str, obj: str, extra=()) -> None:
    cmd = [HIPCC] + CFLAGS + list(extra) + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    msg = _filter(p.stdout)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (os.path.basename(src), msg))
    if msg.strip():
        sys.stderr.write(msg + "\n")


def build(force: bool = False, jobs: int | None = None, verbose: bool = True, variant: str = "") -> str:
    extra, bdir, lname = VARIANTS[variant]
    BUILD = os.path.join(PKG, bdir)
    LIB = os.path.join(PKG, lname)
    os.makedirs(BUILD, exist_ok=True)
    deps_mtime = max(os.path.getmtime(d) for d in _deps())
    todo = []
    objs = []
    for src in _sources():
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        objs.append(obj)
        if force or not os.path.exists(obj) or \
                os.path.getmtime(obj) < max(os.path.getmtime(src), deps_mtime):
            todo.append((src, obj))
    jobs = jobs or min(16, os.cpu_count() or 4)
    if todo:
        if verbose:
            print("[build] compiling %d file(s) with %d job(s)" % (len(todo), jobs), flush=True)
        with cf.ThreadPoolExecutor(jobs) as ex:
            futs = [ex.submit(_compile, s, o, extra) for s, o in todo]
            for f in futs:
                f.result()
    if todo or force or not os.path.exists(LIB):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
        p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if p.returncode != 0:
            raise RuntimeError("link failed:\n" + _filter(p.stdout))
        os.replace(tmp, LIB)
        if verbose:
            print("[build] wrote " + LIB, flush=True)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("--variant", default="", choices=sorted(VARIANTS))
    a = ap.parse_args()
    build(force=a.force, jobs=a.j, variant=a.variant)


if __name__ == "__main__":
    main()
