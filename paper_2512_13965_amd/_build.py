"""Builds libgmc.so (HIP kernels + C ABI) in-tree with hipcc for gfx950."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libgmc.so")
BUILD = os.path.join(PKG, "_build")

SOURCES = ["gmc_mlp.hip", "gmc_film.hip", "gmc_walk.hip", "gmc_transport.hip", "gmc_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-mcode-object-version=5",
         # never emit packed FP32 arithmetic (v_pk_{add,mul,fma}_f32)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
# Per-source device flags.  The samplers' MFMA accumulators stay in ordinary vector registers:
# the four-wave kernels (width 128, FP32) otherwise keep them in accumulation registers and move
# every value out with one extra vector instruction in the epilogue (width 128: 7-8 % of the
# launch); the two-group kernels already keep them there and compile to the same code.
SOURCE_FLAGS = {"gmc_mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"],
                "gmc_film.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def _compile(src: str) -> str:
    out = os.path.join(BUILD, os.path.basename(src) + ".o")
    extra = SOURCE_FLAGS.get(src, [])
    cmd = [HIPCC, *FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and extra and "Unknown command line argument" in r.stdout + r.stderr:
        # a compiler without the register-form option: the same kernels, one more move per value
        print(f"{src}: compiler rejects {' '.join(extra)}; building without it", file=sys.stderr)
        cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and "hip-link" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{errs}")
    if errs.strip():
        print(errs, file=sys.stderr)
    return out


# Host-code sanitizer build (CPU checks only): AddressSanitizer and UndefinedBehaviorSanitizer
# on the host side of every source, device code unchanged.  Loaded by the CPU tests with the
# compiler's ASan runtime preloaded; never shipped as the product library.
ASAN_LIB = os.path.join(BUILD, "libgmc_asan.so")
ASAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def asan_runtime() -> str:
    """Path of the compiler's shared AddressSanitizer runtime (to preload)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "lib", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    return subprocess.check_output([clang, "--print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()


def _compile_asan(src: str) -> str:
    out = os.path.join(BUILD, "asan_" + os.path.basename(src) + ".o")
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"] + ASAN_HOST
    r = subprocess.run([HIPCC, *flags, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc (sanitizer build) failed for {src}:\n{r.stdout}{r.stderr}")
    return out


def build_asan() -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile_asan, srcs))
    tmp = ASAN_LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *ASAN_HOST[:4],
                        "-Xarch_host", "-shared-libsan", "-o", tmp, *objs], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitizer link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, ASAN_LIB)
    return ASAN_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
