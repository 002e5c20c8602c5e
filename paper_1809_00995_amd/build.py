"""Build ``libah.so`` (the gfx950 HIP library behind include/ah.h) in-tree.

Runs ``hipcc --offload-arch=gfx950`` on four translation units -- the C ABI
with every other kernel (``csrc/ah_api.hip``), the FP32 two-steps-per-pass
kernels (``csrc/k_step_tiled2_f32.hip``), and the FP64 ones of one realization
(``csrc/k_step_tiled2_f64.hip``) and of many (``csrc/k_step_batch2_f64.hip``)
-- in parallel, then links them.
Packed-FP32 instruction selection is switched off for all device code
(``-Xclang -target-feature -Xclang -packed-fp32-ops``).  The two-step kernels
take machine schedulers that favour instruction-level parallelism, measured
on one GPU against the default: FP32 ``max-ilp`` (pairs 2.4 % faster), FP64
``iterative-ilp`` for one realization (1.9 % faster; ``max-ilp`` made them
0.8 % slower).  The batched FP64 pair kernel keeps the default (it spills 29
VGPRs there, 41 with ``iterative-ilp``), and so do the single-step kernels,
which holds their occupancy (with ``max-ilp`` the batched one takes 130
instead of 95 VGPRs, 3 instead of 5 waves per SIMD).
"""
from __future__ import annotations

import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
# translation unit -> extra hipcc options
UNITS = [("ah_api.hip", []),
         ("k_step_tiled2_f32.hip", ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]),
         ("k_step_tiled2_f64.hip", ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]),
         ("k_step_batch2_f64.hip", [])]
LIB = os.path.join(PKG, "libah.so")
ARCH = "gfx950"
# options of every unit's device and host code (include paths aside)
COMMON = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def unit_options(src: str) -> list:
    """The hipcc options a translation unit is compiled with (include paths aside)."""
    return COMMON + dict(UNITS)[src]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return exe


def build(verbose: bool = False) -> str:
    incl = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    for src, _ in UNITS:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc()] + unit_options(src) + incl + ["-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    failed = [src for p, src in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc " + " ".join(failed))
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    for obj in objs:
        os.remove(obj)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
