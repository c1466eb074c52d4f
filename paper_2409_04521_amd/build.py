"""Compile the HIP library libfrt.so for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfrt.so")
SOURCES = ["frt_kernels.hip", "frt_merge.hip", "frt_microbench.hip", "frt_engine.cpp", "frt_server.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


# host code checked by AddressSanitizer and UBSan (the device code is built
# as usual: every -fsanitize is for the host side only)
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Xarch_host", "-g"]
HOST_SOURCES = ["frt_engine.cpp", "frt_server.cpp"]


def build_host_sanitized(out: str, verbose: bool = False) -> str:
    """A copy of the library whose host code (engine, serving layer) is built
    with AddressSanitizer and UBSan, linked with the kernel objects of the
    last build().  Load it with the sanitizer runtime preloaded and name it
    in FRT_LIB."""
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        if src in HOST_SOURCES:
            obj = os.path.join(os.path.dirname(out), os.path.splitext(src)[0] + ".san.o")
            cmd = [HIPCC, *FLAGS, *HOST_SANITIZE, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd, stderr=None if verbose else subprocess.DEVNULL)
        elif not os.path.exists(obj):
            raise FileNotFoundError(f"{obj} is missing: run build() first")
        objs.append(obj)
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out])
    return out


def sanitizer_runtime() -> str:
    """The AddressSanitizer runtime of hipcc's host compiler (to preload)."""
    res = subprocess.check_output([os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang"),
                                   "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    if not os.path.isabs(res) or not os.path.exists(res):
        raise FileNotFoundError("no AddressSanitizer runtime next to hipcc's clang")
    return res


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC, *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, stderr=None if verbose else subprocess.DEVNULL)
        objs.append(obj)
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    if "--host-sanitized" in sys.argv:
        print(build_host_sanitized(sys.argv[sys.argv.index("--host-sanitized") + 1], verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
