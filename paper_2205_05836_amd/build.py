"""Builds libcutqc.so (HIP kernels for gfx950 + the C ABI) in this directory.

    python -m paper_2205_05836_amd.build

Every source is compiled with hipcc; packed-FP32 instructions are disabled
for all device code.  The device assembly of gemm.hip is kept (in _build/)
and checked by check_asm against the LDS-DMA counts its hand-counted waits
assume; the build fails when it does not hold.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcutqc.so")
ARCH = "gfx950"
ASM_CHECKED = ("gemm.hip",)


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


def _device_asm(name: str) -> str:
    """The gfx950 assembly hipcc keeps for source `name` (-save-temps=obj)."""
    return os.path.join(BUILD, f"{name[:name.rindex('.')]}-hip-amdgcn-amd-amdhsa-{ARCH}.s")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if os.path.basename(src) in ASM_CHECKED and os.path.exists(_device_asm(os.path.basename(src))):
        os.remove(_device_asm(os.path.basename(src)))  # never check a stale one
    cmd = [hipcc(), "-c", src, "-o", obj, "-O3", "-fPIC", "-std=c++17",
           f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC, "-Wall",
           "-Wno-unused-function", "-Wno-unused-variable"]
    if src.endswith(".hip"):
        cmd += ["-x", "hip", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics"]
    if os.path.basename(src) in ASM_CHECKED:
        cmd += ["-save-temps=obj"]  # keeps the device assembly next to the object
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    from . import check_asm
    for name in ASM_CHECKED:
        path = _device_asm(name)
        if not os.path.exists(path):
            raise RuntimeError(f"device assembly of {name} not found in {BUILD}")
        errs = check_asm.check(path)
        if errs:
            raise RuntimeError("assembly check failed:\n" + "\n".join(errs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
