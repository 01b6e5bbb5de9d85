"""Build the HIP library ``libdcdft.so`` in-tree for gfx950.

Every source under ``csrc/`` is compiled with hipcc (one object per file, in
parallel) and linked into a shared library next to this file.  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdcdft.so")
ARCH = os.environ.get("DCDFT_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ROCM_LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "lib")
# roctx ranges of the runtime (marker traces of rocprofv3); rocBLAS and rocSOLVER
# for the dense algebra of the large-orbital path
LIBS = [f"-L{ROCM_LIB}", "-lrocprofiler-sdk-roctx", "-lrocsolver", "-lrocblas"]
CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-Wno-unused-result"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{res.stderr[-6000:]}")
    return obj


# host-side AddressSanitizer and UndefinedBehaviorSanitizer for the runtime
# (api.hip): each -fsanitize= applies to the host pass only, the device code is
# built as usual
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-shared-libasan"]
SAN_LIB = os.path.join(BUILD, "san", "libdcdft_san.so")


def asan_runtime() -> str:
    """Path of the shared AddressSanitizer runtime of the ROCm compiler (to be
    preloaded into a process that loads the sanitized library), or ''."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "lib", "llvm", "bin",
                         "clang")
    if not os.path.exists(clang):
        clang = shutil.which("clang") or "/opt/rocm/llvm/bin/clang"
    res = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = res.stdout.strip()
    return path if res.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else ""


def build_host_sanitized() -> str:
    """The library with its host runtime (api.hip) built under the sanitizers and
    the kernel objects of the regular build (built first if missing); for the
    host-only ABI checks."""
    objs = [os.path.join(BUILD, os.path.basename(s)[:-4] + ".o") for s in sources()
            if not s.endswith("api.hip")]
    if not all(os.path.exists(o) for o in objs):
        build()
    os.makedirs(os.path.dirname(SAN_LIB), exist_ok=True)
    api_obj = os.path.join(os.path.dirname(SAN_LIB), "api_san.o")
    cmd = [HIPCC, "-O1", "-g", *[f for f in CFLAGS if f != "-O3"], *SAN_FLAGS, "-c",
           os.path.join(CSRC, "api.hip"), "-o", api_obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on api.hip:\n{res.stderr[-6000:]}")
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", api_obj, *objs, *SAN_FLAGS,
           *LIBS, "-o", SAN_LIB]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-6000:]}")
    return SAN_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, *LIBS, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
