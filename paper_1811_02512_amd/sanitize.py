"""CPU sanitizer check of the host code: libpf (host analysis, symbolic
handles, argument checking and every other host path of the C ABI) and the
oracle built with AddressSanitizer and UndefinedBehaviorSanitizer, then the
CPU test suite (pytest -m "not gpu") run against those builds.

Device code is compiled as usual: every sanitizer flag on a hipcc line is
scoped to the host pass.  The instrumented libraries go to _build/sanitize/;
the run selects them with PF_LIBPF / PF_LIBORACLE and preloads the sanitizer
runtime of the compiler that built them (Python itself is not
instrumented).  Usage, from the repository root:
    python paper_1811_02512_amd/sanitize.py [extra pytest arguments]
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
sys.path.insert(0, PKG)

import build as B  # noqa: E402  (the regular build's sources and flags)

OUT = os.path.join(B.BUILD, "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
            "-fno-omit-frame-pointer"]


def runtime():
    libs = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not libs:
        raise RuntimeError("no clang AddressSanitizer runtime under /opt/rocm/llvm")
    return sorted(libs)[-1]


def build() -> tuple:
    os.makedirs(OUT, exist_ok=True)
    objs = []
    flags = [f for f in B.COMMON if f != "-O3"] + ["-O1", "-g"]
    for src in ("analyze.cpp",):
        obj = os.path.join(OUT, src + ".o")
        B._run([B.HIPCC, *flags, *HOST_SAN, "-c", os.path.join(B.CSRC, src), "-o", obj])
        objs.append(obj)
    for src in B.KERNEL_FILES:
        obj = os.path.join(OUT, src + ".o")
        B._run([B.HIPCC, *flags, *B.DEVICE_FLAGS, *HOST_SAN, "-c", os.path.join(B.CSRC, src),
                "-o", obj])
        objs.append(obj)
    lib = os.path.join(OUT, "libpf.so")
    B._run([B.HIPCC, "-shared", "-fPIC", *B.DEVICE_FLAGS, *HOST_SAN, "-Xarch_host",
            "-shared-libasan", "-o", lib, *objs])
    olib = os.path.join(OUT, "liboracle.so")
    san_c = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-shared-libasan"]
    B._run([CLANG, "-O1", "-g", "-std=gnu99", "-fPIC", "-shared", *san_c, "-o", olib,
            os.path.join(ROOT, "oracle", "pf_oracle.c"), "-lm"])
    return lib, olib


def main(argv):
    lib, olib = build()
    env = dict(os.environ)
    env.update(PF_LIBPF=lib, PF_LIBORACLE=olib, LD_PRELOAD=runtime(),
               ASAN_OPTIONS="detect_leaks=0:alloc_dealloc_mismatch=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    print(f"[sanitize] libpf {lib}\n[sanitize] oracle {olib}\n[sanitize] runtime {runtime()}",
          flush=True)
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "tests", *argv]
    return subprocess.call(cmd, cwd=ROOT, env=env)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
