"""Build the gfx950 HIP library libmagpie.so in-tree with hipcc.

Run as ``python -m paper_2504_10118_amd.build``.  Packed FP32 instructions
are disabled for all device code (``-target-feature -packed-fp32-ops``).

``build_asan_driver()`` links the same sources with ``tests/asan_driver.cpp``
into one executable whose host code (the C ABI, its runtime and the kernel
launchers) carries AddressSanitizer; device code is built as usual.

Each source is compiled to an object of its own, in parallel, and hipcc then
links the objects (one hipcc command that mixes HIP and C++ sources loses the
offload architecture, and one object per source keeps the build short).
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libmagpie.so")
ASAN_DRIVER = os.path.join(LIBDIR, "magpie_asan_driver")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["kernels.hip", "cnn.hip", "capi.cpp", "learned.cpp", "noalloc.hip"]
ARCH = os.environ.get("MAGPIE_OFFLOAD_ARCH", "gfx950")
ASAN_FLAGS = ["-gline-tables-only", "-Xarch_host", "-fsanitize=address",
              "-Xarch_host", "-fno-omit-frame-pointer"]


def hipcc_path() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def _compile_flags() -> list:
    return [hipcc_path(), f"--offload-arch={ARCH}", "-O3", "-std=c++17",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd: list, tmp: str, out: str, verbose: bool) -> str:
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}")
    os.replace(tmp, out)
    return out


def _objects(jobs: list, verbose: bool) -> None:
    """jobs: (source, language, extra flags, object path); compiled concurrently."""
    def one(job):
        src, lang, extra, obj = job
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        return _run(_compile_flags() + extra + ["-c", "-x", lang, src, "-o", obj + ".tmp"],
                    obj + ".tmp", obj, verbose)
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1, 8)) as ex:
        list(ex.map(one, jobs))


def _lib_jobs() -> list:
    return [(os.path.join(CSRC, s), "hip", ["-fPIC"], os.path.join(OBJDIR, "lib", s + ".o"))
            for s in SOURCES]


def _asan_jobs() -> list:
    jobs = [(os.path.join(CSRC, s), "hip", ASAN_FLAGS, os.path.join(OBJDIR, "asan", s + ".o"))
            for s in SOURCES]
    jobs.append((os.path.join(ROOT, "tests", "asan_driver.cpp"), "c++", ASAN_FLAGS,
                 os.path.join(OBJDIR, "asan", "asan_driver.cpp.o")))
    return jobs


def _link_lib(verbose: bool) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc_path(), f"--offload-arch={ARCH}", "-shared", "-fPIC"] + [j[3] for j in _lib_jobs()]
    return _run(cmd + ["-o", tmp], tmp, LIB, verbose)


def _link_asan(verbose: bool) -> str:
    tmp = ASAN_DRIVER + ".tmp"
    cmd = [hipcc_path(), f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address"]
    cmd += [j[3] for j in _asan_jobs()]
    return _run(cmd + ["-o", tmp], tmp, ASAN_DRIVER, verbose)


def build(verbose: bool = False, asan_driver: bool = False) -> str:
    """libmagpie.so (and, with asan_driver, the AddressSanitizer executable, built
    alongside).  Returns the library's path."""
    os.makedirs(LIBDIR, exist_ok=True)
    _objects(_lib_jobs() + (_asan_jobs() if asan_driver else []), verbose)
    if asan_driver:
        _link_asan(verbose)
    return _link_lib(verbose)


def build_asan_driver(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    _objects(_asan_jobs(), verbose)
    return _link_asan(verbose)


if __name__ == "__main__":
    print(build(verbose=True, asan_driver="--asan" in sys.argv))
