"""Build libbs.so (hand-written HIP for gfx950) in-tree with hipcc.

Every HIP source under csrc/ is compiled to an object file (in parallel, one
hipcc process per source; no relocatable device code: each source holds all
the device code its kernels call) and the objects are linked into one shared
library next to this file.  Packed-FP32 instructions are disabled for device
code (the compiler would otherwise form v_pk_* FP32 operations from scalar
code).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbs.so")
ARCH = os.environ.get("BS_OFFLOAD_ARCH", "gfx950")

FLAGS = [f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def compile_command(src: str, obj: str):
    return (["hipcc"] + FLAGS + ["-I", os.path.join(ROOT, "include"),
                                 "-I", os.path.join(HERE, "csrc"), "-c", src, "-o", obj])


def link_command(objs, out: str = LIB):
    return ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + list(objs) + \
        ["-lhipfft"]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(os.cpu_count() or 1, 16)))
    with tempfile.TemporaryDirectory(prefix="bs_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.basename(s) + ".o") for s in srcs]

        def one(i):
            cmd = compile_command(srcs[i], objs[i])
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, capture_output=True, text=True)

        with ThreadPoolExecutor(jobs) as ex:
            res = list(ex.map(one, range(len(srcs))))
        bad = [r for r in res if r.returncode != 0]
        for r in res:
            # the host pass does not know the device-only feature flag
            msg = "".join(ln for ln in (r.stdout + r.stderr).splitlines(True)
                          if "packed-fp32-ops' is not a recognized feature" not in ln)
            if msg:
                sys.stderr.write(msg)
        if bad:
            raise RuntimeError("hipcc failed building libbs.so")
        tmp = LIB + ".tmp"
        cmd = link_command(objs, tmp)
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libbs.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
