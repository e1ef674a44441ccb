"""Build libp2m.so (all HIP sources, gfx950) in-tree.

Usage: python -m paper_1610_05266_amd.build [--jobs N] [--debug]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libp2m.so")
ARCH = os.environ.get("P2M_OFFLOAD_ARCH", "gfx950")

SOURCES = ["util.hip", "binning.hip", "build.hip", "project.hip", "m2p.hip", "adjoint.hip", "transpose.hip",
           "advect.hip", "profile.hip", "capi.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libp2m)")


def flags(debug: bool):
    f = [
        f"--offload-arch={ARCH}",
        "-std=c++17",
        "-fPIC",
        "-O1" if debug else "-O3",
        "-munsafe-fp-atomics",
        # packed FP32 instructions off
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE,
        "-I", CSRC,
        "-Wall",
        "-Wno-unused-function",
        # a self-call left in a device helper is an endless loop the optimiser
        # may delete together with everything after it
        "-Werror=infinite-recursion",
        "-Werror=uninitialized",
    ]
    return f


def device_asm(src: str, out: str, debug: bool = False) -> str:
    """gfx950 assembly of one source (device pass only), for inspection."""
    cmd = [hipcc(), *flags(debug), "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"device compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


def compile_one(src: str, debug: bool) -> str:
    out = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *flags(debug), "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    # the host pass does not know the packed-fp32 feature; that warning is harmless
    msg = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l and l.strip())
    if msg.strip():
        sys.stderr.write(msg + "\n")
    return out


def build(jobs: int = 8, debug: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(lambda s: compile_one(s, debug), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


# sources whose host code the sanitizer build instruments: the C ABI's
# argument checks, handles and workspaces (the rest is linked as built)
ASAN_SOURCES = ["capi.hip", "util.hip", "profile.hip"]
ASAN_DIR = os.path.join(OBJDIR, "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libp2m_asan.so")


def asan_runtime() -> str:
    """Path of the compiler's shared AddressSanitizer runtime."""
    r = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("the AddressSanitizer runtime of the HIP compiler was not found")
    return path


def build_host_asan(jobs: int = 8) -> str:
    """libp2m with AddressSanitizer in the host code of ASAN_SOURCES (device
    code and the other sources as in build()), for checking the C ABI's host
    paths on a CPU; load it with the runtime from asan_runtime() preloaded."""
    os.makedirs(ASAN_DIR, exist_ok=True)
    host_asan = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]

    def one(src: str) -> str:
        if src in ASAN_SOURCES:
            out = os.path.join(ASAN_DIR, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc(), *flags(False), *host_asan, "-c", os.path.join(CSRC, src), "-o", out]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
            return out
        out = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        return out if os.path.exists(out) else compile_one(src, False)

    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(one, SOURCES))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-shared-libsan", *objs, "-o", ASAN_LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return ASAN_LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.debug))


if __name__ == "__main__":
    main()
