"""Build liboras.so (HIP, gfx950) in-tree.

    python -m paper_2110_15113_amd.build          # or build() from Python
    python -m paper_2110_15113_amd.build --asan   # host code under AddressSanitizer

Compiles every source under csrc/ with hipcc for gfx950 and links
paper_2110_15113_amd/liboras.so.  Objects go to paper_2110_15113_amd/_build/.

--asan instruments the host code only (-Xarch_host -fsanitize=address; the
device code is unchanged) and links paper_2110_15113_amd/_build_asan/
liboras.so.  Load it into a process started with the sanitizer runtime
preloaded (asan_runtime() gives its path) and ORAS_LIB pointing at it.
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
LIB = os.path.join(HERE, "liboras.so")
ARCH = os.environ.get("ORAS_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(HERE, "..", "include"),
]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


ASAN_BUILD = os.path.join(HERE, "_build_asan")
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """Path of the AddressSanitizer runtime of the ROCm clang."""
    clang = os.path.join(os.path.dirname(os.path.realpath(_hipcc())), "..", "lib", "llvm", "bin",
                         "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                       text=True)
    return r.stdout.strip()


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, src + ".o")
    cmd = [_hipcc(), *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".hip"):
        cmd.insert(1, "-xhip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, asan: bool = False) -> str:
    build_dir = ASAN_BUILD if asan else BUILD
    lib = os.path.join(ASAN_BUILD, "liboras.so") if asan else LIB
    extra = ASAN_FLAGS if asan else []
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, build_dir, extra), srcs))
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", f"--offload-arch={ARCH}", *extra, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    try:
        build(verbose=True, asan="--asan" in sys.argv[1:])
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
