"""Builds libptyg.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

    python -m paper_2106_07575_amd.build              # or build() from Python
    python -m paper_2106_07575_amd.build --sanitize   # host-sanitizer variant

The sanitizer variant (_build/sanitize/libptyg.so) instruments the host
code only (AddressSanitizer and UndefinedBehaviorSanitizer on the host
pass; device code is built as usual) for the CPU-side tests; a process
loads it with the ASan runtime preloaded (asan_runtime()).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libptyg.so")
BUILD = os.path.join(PKG, "_build")
SOURCES = ["kernels.hip", "kernels256.hip", "nn.hip", "api.hip"]
ARCH = os.environ.get("PTYG_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in any HIP code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware float atomics for the scatter-add
    "-munsafe-fp-atomics",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libptyg.so)")


SAN_BUILD = os.path.join(BUILD, "sanitize")
SAN_LIB = os.path.join(SAN_BUILD, "libptyg.so")
# host pass only: each -fsanitize= goes to the host compiler
SAN_FLAGS = ["-O1", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, sanitize: bool = False) -> str:
    out = SAN_BUILD if sanitize else BUILD
    obj = os.path.join(out, os.path.splitext(src)[0] + ".o")
    flags = [f for f in FLAGS if f != "-O3"] + SAN_FLAGS if sanitize else FLAGS
    cmd = [hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = True, sanitize: bool = False) -> str:
    """Compile every HIP source and link libptyg.so next to this file (the
    sanitizer variant: under _build/sanitize)."""
    out, lib = (SAN_BUILD, SAN_LIB) if sanitize else (BUILD, LIB)
    os.makedirs(out, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), SOURCES))
    tmp = lib + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}", file=sys.stderr)
    return lib


def sources_newer_than(path: str) -> bool:
    """True when `path` is missing or older than a source or header."""
    if not os.path.exists(path):
        return True
    t = os.path.getmtime(path)
    inc = os.path.join(os.path.dirname(PKG), "include")
    files = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.join(inc, f) for f in os.listdir(inc)]
    return any(os.path.getmtime(f) > t for f in files)


def asan_runtime() -> str:
    """The AddressSanitizer runtime of the compiler hipcc drives."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = shutil.which("clang++") or "clang++"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("AddressSanitizer runtime not found")
    return path


if __name__ == "__main__":
    build(sanitize="--sanitize" in sys.argv[1:])
