"""Build libsv.so (HIP kernels for gfx950 + host C ABI) in-tree.

    python paper_2409_14697_amd/build.py        # or __graft_entry__.build()

Every source under csrc/ is compiled with hipcc for gfx950 and linked into
paper_2409_14697_amd/libsv.so.  Packed FP32 instructions are disabled for the
device code (-packed-fp32-ops).

SV_SANITIZE=1 builds a debug variant instead, _build/sanitize/libsv.so: the
host-only sources (the C ABI, planners, packer, batcher: compiled with g++)
carry UndefinedBehaviorSanitizer, aborting on the first report; device code
is unchanged.  Load it with SV_LIBRARY=<path> to run the CPU tests under it:

    SV_SANITIZE=1 python paper_2409_14697_amd/build.py
    SV_SANITIZE=1 SV_LIBRARY=_build/sanitize/libsv.so python -m pytest tests -m "not gpu"

(the host model of the tile-pass kernel, tests/emu, is then built with
AddressSanitizer as well).
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
SANITIZE = os.environ.get("SV_SANITIZE", "") not in ("", "0")
BUILD = os.path.join(ROOT, "_build", "sanitize") if SANITIZE else os.path.join(ROOT, "_build")
LIB = os.path.join(BUILD, "libsv.so") if SANITIZE else os.path.join(PKG, "libsv.so")
HOST_SANITIZE = ["-g", "-fsanitize=undefined", "-fno-sanitize-recover=undefined"] if SANITIZE else []

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.environ.get("HIPCC", f"{ROCM}/bin/hipcc")
CXX = os.environ.get("SV_CXX", "g++")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def sources():
    out = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith(".hip") or f.endswith(".cpp"):
            out.append(os.path.join(CSRC, f))
    return out


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC] + COMMON + ["-x", "hip"] + DEVICE
    else:  # host-only C++: plain g++ against the HIP runtime headers
        cmd = [CXX] + COMMON + HOST_SANITIZE + ["-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]
    cmd += ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn.strip() and "warning" in warn:
        sys.stderr.write(warn + "\n")
    return obj


def build(verbose: bool = True) -> str:
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs + [f"-L{ROCM}/lib", "-lamdhip64"]
    if SANITIZE:
        cmd.append("-lubsan")  # the runtime of the host objects' checks
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
