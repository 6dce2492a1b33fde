"""AddressSanitizer + UndefinedBehaviorSanitizer build of the library's host
code, for CPU tests of the host calls.

The host-only sources (parameters, key generation, encryption, decryption,
planning and packing) are compiled with the sanitizers on the host pass only;
the HIP sources are the ordinary objects of ``build.py``. The result,
``_build/asan/libhyena.so``, is loaded instead of the in-tree library by
setting ``HYENA_LIB`` and preloading the sanitizer runtime (``run_tests``).
GPU code is never built with a sanitizer.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

from . import build as hb

HOST_SOURCES = ["params.cpp", "crypto.cpp", "plan.cpp"]
OUT_DIR = os.path.join(hb.BUILD_DIR, "asan")
OUT = os.path.join(OUT_DIR, "libhyena.so")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def runtime() -> str:
    """The clang AddressSanitizer runtime that hipcc links against."""
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not libs:
        raise RuntimeError("clang AddressSanitizer runtime not found under /opt/rocm/llvm")
    return libs[-1]


def build() -> str:
    hb.build()                      # the ordinary objects (HIP sources) in _build/
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    for src in hb.SOURCES:
        if src in HOST_SOURCES:
            obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
            flags = [f for f in hb.FLAGS if f != "-O3"] + ["-O1", "-g"] + SAN
            cmd = [hb.HIPCC, *flags, "-c", "-x", "hip", os.path.join(hb.CSRC, src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"sanitizer build of {src} failed:\n{r.stderr}")
            objs.append(obj)
        else:
            objs.append(os.path.join(hb.BUILD_DIR, os.path.splitext(src)[0] + ".o"))
    vs = os.path.join(hb.BUILD_DIR, "exports.map")
    cmd = [hb.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", OUT, *objs, "-lpthread",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan",
           "-Wl,--version-script=" + vs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitizer link failed:\n{r.stderr}")
    return OUT


def run_tests(tests=("tests/test_host_abi.py",), timeout: int = 600) -> subprocess.CompletedProcess:
    """Run CPU tests of the host calls against the sanitizer build in a child
    process (the runtime must be preloaded before Python starts)."""
    env = dict(os.environ)
    env["HYENA_LIB"] = OUT
    env["LD_PRELOAD"] = runtime()
    # CPython itself keeps memory at exit; leaks are not what this run checks
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                           "-p", "no:cacheprovider", *tests],
                          cwd=hb.ROOT, env=env, capture_output=True, text=True, timeout=timeout)


if __name__ == "__main__":
    print("built", build())
    r = run_tests()
    sys.stdout.write(r.stdout[-3000:])
    sys.stderr.write(r.stderr[-3000:])
    sys.exit(r.returncode)
