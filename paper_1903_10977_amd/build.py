"""In-tree build of the native libraries.

libimsmg.so      HIP solver library for gfx950 (hipcc)
libimsmg_gen.so  host C++ problem generator (g++ / OpenMP)

Both are rebuilt on every call of build_all(); tests, smoke and the bench load
what is built and fail loudly when it is missing.
"""
from __future__ import annotations

import os
import subprocess
import sys

from . import INCLUDE_DIR, LIB_DIR, PACKAGE_DIR

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# packed FP32 instructions are disabled for every HIP translation unit
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=fast", "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
             "-Wno-unused-variable", "-Wno-unused-but-set-variable"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r.stdout


def build_generator() -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    out = os.path.join(LIB_DIR, "libimsmg_gen.so")
    src = os.path.join(PACKAGE_DIR, "gen", "generator.cpp")
    _run(["g++", "-O3", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
          "-I", INCLUDE_DIR, "-o", out + ".tmp", src])
    os.replace(out + ".tmp", out)
    return out


def hip_sources():
    d = os.path.join(PACKAGE_DIR, "csrc")
    return sorted(os.path.join(d, f) for f in os.listdir(d) if f.endswith(".hip"))


def build_solver() -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    out = os.path.join(LIB_DIR, "libimsmg.so")
    srcs = hip_sources()
    if not srcs:
        raise RuntimeError("no HIP sources")
    _run([HIPCC] + HIP_FLAGS + ["-I", INCLUDE_DIR, "-o", out + ".tmp"] + srcs)
    os.replace(out + ".tmp", out)
    return out


def build_all():
    return build_generator(), build_solver()


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("gen", "all"):
        print(build_generator())
    if what in ("solver", "all"):
        print(build_solver())
