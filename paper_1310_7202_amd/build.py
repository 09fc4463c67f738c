"""Build librlu.so (the HIP kernels and the C ABI) for gfx950, in-tree.

    python -m paper_1310_7202_amd.build             # or build() from Python
    python -m paper_1310_7202_amd.build sanitized   # host code under ASan + UBSan

Every call recompiles.  Objects go to ``_build/`` at the repository root,
the shared library to ``paper_1310_7202_amd/librlu.so``.  The sanitized
variant (``_build/librlu_san.so``) instruments the host translation units
(the C ABI, the batch planner and the server) with AddressSanitizer and
UndefinedBehaviorSanitizer and links them with the ordinary kernel objects;
it is for the CPU tests of the ABI, loaded into a process that preloads the
sanitizer runtime (``sanitizer_runtime()``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librlu.so")

ARCH = "gfx950"
# Packed FP32 instructions are disabled on purpose (no v_pk_* FP32 math).
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}",
]

SOURCES = ["rng.hip", "gemm.hip", "gemm_lp.hip", "gemm_lp_stream.hip", "panel_lu.hip",
           "spd_inverse.hip", "finish.hip", "lstsq.hip", "rrlu.hip", "fast_lu.hip",
           "rlu_api.cpp", "rlu_batch.cpp", "rlu_serve.cpp"]
HOST_SOURCES = [s for s in SOURCES if s.endswith(".cpp")]
SAN_LIB = os.path.join(BUILD_DIR, "librlu_san.so")
# sanitizers for the host pass only (the device code is built as usual)
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build librlu)")


def _compile(src: str, hipcc: str, extra=(), suffix=".o") -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + suffix)
    cmd = [hipcc, "-x", "hip", *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    workers = min(len(SOURCES), max(1, (os.cpu_count() or 2) // 2), 8)
    with cf.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(lambda s: _compile(s, hipcc), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


def sanitizer_runtime() -> str:
    """Path of the shared AddressSanitizer runtime of the HIP compiler."""
    import glob
    root = os.path.dirname(os.path.dirname(os.path.realpath(_hipcc())))
    for base in (os.path.join(root, "llvm"), "/opt/rocm/llvm"):
        hits = sorted(glob.glob(os.path.join(base, "lib", "clang", "*", "lib", "linux",
                                             "libclang_rt.asan-x86_64.so")))
        if hits:
            return hits[-1]
    raise RuntimeError("libclang_rt.asan-x86_64.so not found")


def build_sanitized(verbose: bool = False) -> str:
    """_build/librlu_san.so: the host sources under ASan + UBSan, the kernel
    objects as in build() (compiled here if they are missing)."""
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    kernels = [s for s in SOURCES if s not in HOST_SOURCES]
    objs = []
    for src in kernels:
        obj = os.path.join(BUILD_DIR, src + ".o")
        objs.append(obj if os.path.exists(obj) else _compile(src, hipcc))
    with cf.ThreadPoolExecutor(len(HOST_SOURCES)) as ex:
        objs += list(ex.map(lambda s: _compile(s, hipcc, ("-O1", "-g", *SAN_FLAGS), ".san.o"),
                            HOST_SOURCES))
    tmp = SAN_LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan", *SAN_FLAGS,
           *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, SAN_LIB)
    if verbose:
        print(f"built {SAN_LIB}")
    return SAN_LIB


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "sanitized":
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
