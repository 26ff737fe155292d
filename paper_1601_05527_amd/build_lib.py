"""Compile libad.so (hand-written HIP for gfx950) in-tree.

    python -m paper_1601_05527_amd.build_lib
    python -m paper_1601_05527_amd.build_lib --sanitize

The second form builds _build_san/libad_san.so: the same sources at -O1
with AddressSanitizer and UndefinedBehaviorSanitizer on the host code only
(device code is not instrumented); it runs the host-side logic -- argument
checks, workspace carving, launch planning -- under the sanitizers, with
clang's ASan runtime preloaded into the process (sanitizer_runtime()).

Each ``csrc/*.hip`` file is compiled to an object with hipcc in parallel,
then linked into ``paper_1601_05527_amd/libad.so``.  The measurement probe
``probe/gather_probe.hip`` (a pure row-gather kernel the benchmark uses as a
ceiling, not part of the method) becomes ``libad_probe.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libad.so")
PROBE_SRC = os.path.join(HERE, "probe", "gather_probe.hip")
PROBE_LIB = os.path.join(HERE, "libad_probe.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
# Packed FP32 instructions stay disabled for all device code.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-function"]


SAN_BUILD = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_BUILD, "libad_san.so")
# host-side sanitizers only: each flag goes to the host compilation
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _compile(src: str, out_dir: str = BUILD, flags=None) -> str:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC] + (FLAGS if flags is None else flags) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def sanitizer_runtime() -> str:
    """Path of the ASan runtime of the HIP compiler (to preload into a
    process that loads the sanitized library)."""
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise RuntimeError("no clang ASan runtime found under /opt/rocm/llvm")
    return found[-1]


def build_sanitized(verbose: bool = False) -> str:
    os.makedirs(SAN_BUILD, exist_ok=True)
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"] + SAN_HOST
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s_: _compile(s_, SAN_BUILD, flags), srcs))
    tmp = SAN_LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}"] + SAN_HOST[:4] + objs + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, SAN_LIB)
    if verbose:
        print(f"built {SAN_LIB}")
    return SAN_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}"] + objs + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    tmp = PROBE_LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-shared", PROBE_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {PROBE_SRC}:\n{r.stderr}")
    os.replace(tmp, PROBE_LIB)
    if verbose:
        print(f"built {LIB} and {PROBE_LIB}")
    return LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv[1:]:
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
