"""Builds a copy of libmbdp.so whose host runtime (mbdp_runtime.hip's CPU
code: argument checks, workspace layout, handles, status mapping) carries
AddressSanitizer and UndefinedBehaviorSanitizer, for the CPU boundary
tests.  The device code is not instrumented (GPU sanitizers are not used);
the kernel translation units are the objects of the normal build.

    python -m paper_2110_02901_amd.build_sanitized

Loading the result needs clang's ASan runtime preloaded into the process
(``asan_runtime()``), since the Python interpreter is not instrumented.
"""
import glob
import os
import subprocess
import sys

from . import build

SAN_LIB = os.path.join(build.OBJDIR, "libmbdp_san.so")
# host-only instrumentation: each sanitizer flag applies to the host pass
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-shared-libsan"]


def asan_runtime():
    """Path of clang's shared ASan runtime that the sanitized library links."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cands = sorted(glob.glob(os.path.join(rocm, "llvm", "lib", "clang", "*", "lib", "linux",
                                          "libclang_rt.asan-x86_64.so")))
    if not cands:
        raise RuntimeError("clang's ASan runtime not found under %s" % rocm)
    return cands[-1]


def build_sanitized(verbose=False):
    """Compiles the host runtime with the sanitizers and links it with the
    normal build's kernel objects; returns the library path."""
    os.makedirs(build.OBJDIR, exist_ok=True)
    objs = []
    for src in build.SOURCES:
        if src == "mbdp_runtime.hip":
            continue
        obj = os.path.join(build.OBJDIR, src.replace(".hip", ".o"))
        if not os.path.exists(obj):
            build.build_library(verbose=verbose)
        objs.append(obj)
    san_obj = os.path.join(build.OBJDIR, "mbdp_runtime_san.o")
    cmd = ([build.hipcc()] + build.COMPILE_FLAGS + SANITIZE +
           ["-g", "-I", build.INCLUDE, "-I", build.CSRC, "-c",
            os.path.join(build.CSRC, "mbdp_runtime.hip"), "-o", san_obj])
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("sanitized compile of mbdp_runtime.hip failed")
    cmd = ([build.hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + SANITIZE +
           objs + [san_obj, "-o", SAN_LIB])
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking the sanitized library failed")
    return SAN_LIB


if __name__ == "__main__":
    print(build_sanitized(verbose=True))
