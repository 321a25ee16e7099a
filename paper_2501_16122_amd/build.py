"""Compile the HIP sources of libmapmaker.so for gfx950 (in-tree).

Usage: python -m paper_2501_16122_amd.build   (or __graft_entry__.build())
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmapmaker.so")
ARCH = os.environ.get("MM_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

CFLAGS = [
    "-O3", "-fPIC", "-std=c++20", f"--offload-arch={ARCH}",
    # FP64 atomics compile to hardware global/LDS atomic adds
    "-munsafe-fp-atomics",
    # no packed-FP32 instructions anywhere in the library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-variable", "-Wno-unused-function",
    "-I", INCLUDE, "-I", CSRC,
]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with concurrent.futures.ThreadPoolExecutor(max(1, min(len(srcs), os.cpu_count() or 1, 8))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


# sources whose object the sanitized build takes from the regular build: they
# hold only kernels and their launch wrappers, which no host-only check
# reaches, and their device pass takes minutes
SANITIZE_REUSE = ("toeplitz.hip",)


def build_host_sanitized(out_dir: str) -> str:
    """libmapmaker with its host code under AddressSanitizer and
    UndefinedBehaviorSanitizer (device code built as usual, never run), as
    out_dir/libmapmaker_hostsan.so, for checks of the entry points that need
    no GPU: size queries, option and argument checks, error paths.  The
    objects of SANITIZE_REUSE come unsanitized from the regular build, which
    must exist.  Loading the library needs the compiler's shared ASan
    runtime, e.g. through an executable linked with -fsanitize=address
    -shared-libsan."""
    os.makedirs(out_dir, exist_ok=True)
    reused = [os.path.join(BUILD, s.replace(".hip", ".o")) for s in SANITIZE_REUSE]
    for o in reused:
        if not os.path.exists(o):
            raise FileNotFoundError(f"{o}: run the regular build first")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    flags = [f for f in CFLAGS if f != "-O3"] + ["-O1", "-g", "-fno-omit-frame-pointer", *san]

    def one(src):
        obj = os.path.join(out_dir, src.replace(".hip", ".hostsan.o"))
        cmd = [HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{' '.join(cmd)}\n{r.stderr}")
        return obj

    srcs = [s for s in sources() if s not in SANITIZE_REUSE]
    with concurrent.futures.ThreadPoolExecutor(max(1, min(len(srcs), os.cpu_count() or 1, 8))) as ex:
        objs = list(ex.map(one, srcs))
    lib = os.path.join(out_dir, "libmapmaker_hostsan.so")
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", *san, "-shared-libsan", "-o", lib, *objs, *reused]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stderr}")
    return lib


if __name__ == "__main__":
    build()
