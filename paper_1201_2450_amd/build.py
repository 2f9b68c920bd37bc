"""Build libtnlm.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1201_2450_amd.build   (or call build()).
Every .hip file under csrc/ is compiled to an object in _build/ and the
objects are linked into paper_1201_2450_amd/libtnlm.so. Packed FP32 VALU
instructions are switched off for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libtnlm.so")
ARCH = os.environ.get("TNLM_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"),
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    # hipcc's host pass warns that it does not know the packed-fp32 feature
    noise = "not a recognized feature for this target"
    msgs = [ln for ln in r.stderr.splitlines() if ln.strip() and noise not in ln
            and "ignoring feature" not in ln]
    if msgs:
        sys.stderr.write("\n".join(msgs) + "\n")
    return obj


def _runtime_dir() -> str:
    """Directory of PyTorch's bundled HIP runtime (else the system ROCm's):
    the link records the runtime's SONAME (libamdhip64.so.7), which a torch
    process has already loaded from there."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec and spec.origin:
        d = os.path.join(os.path.dirname(spec.origin), "lib")
        if os.path.exists(os.path.join(d, "libamdhip64.so")):
            return d
    return "/opt/rocm/lib"


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libtnlm.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    # Link against the HIP runtime by its SONAME, so that inside a process
    # that already loaded PyTorch's bundled ROCm runtime the library binds to
    # that same runtime (one HIP/HSA stack per process: device pointers and
    # streams from torch stay valid); standalone it resolves to the system
    # ROCm.
    cmd = ["g++", "-shared", "-fPIC", "-o", tmp, *objs, "-L" + _runtime_dir(),
           "-l:libamdhip64.so", "-Wl,--no-undefined", "-lstdc++", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
