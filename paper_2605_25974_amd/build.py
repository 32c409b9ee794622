"""Builds libpaulisum.so (HIP, gfx950) in place next to this file.

Every source under csrc/ is compiled by hipcc for gfx950 only, with
floating-point contraction off (the plain coefficient product is rounded
operation by operation) and packed-FP32 instructions disabled, then linked
into one shared library that exports the C ABI of include/paulisum.h.
`python build.py --asan` builds a host-side AddressSanitizer variant under
_build/asan/ instead (a checking aid; the package never loads it).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpaulisum.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-I", os.path.join(os.path.dirname(HERE), "include"),
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


# Host-side AddressSanitizer build (a checking aid, never loaded by the
# package): the host code of every unit is instrumented, the device code is
# not.  The library is linked without the sanitizer runtime; a process that
# loads it preloads that runtime (asan_runtime()).
ASAN_DIR = os.path.join(BUILD, "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libpaulisum_asan.so")
ASAN_FLAGS = [f for f in FLAGS if f != "-O3"] + [
    "-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src, flags=None, outdir=None):
    obj = os.path.join(outdir or BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + (flags or FLAGS) + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, r.stderr[-6000:]))
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-6000:])
    os.replace(tmp, lib)
    return lib


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    return _link(objs, LIB)


def build_asan(jobs: int | None = None) -> str:
    """Builds _build/asan/libpaulisum_asan.so with host-side ASan."""
    os.makedirs(ASAN_DIR, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, ASAN_FLAGS, ASAN_DIR), srcs))
    return _link(objs, ASAN_LIB)


def asan_runtime() -> str | None:
    """The compiler's shared ASan runtime (to preload), or None."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


if __name__ == "__main__":
    print(build_asan() if "--asan" in sys.argv[1:] else build())
    sys.exit(0)
