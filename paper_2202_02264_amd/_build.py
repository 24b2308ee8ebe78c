"""Build libdsmc.so (the HIP kernels and the C ABI) in-tree for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libdsmc.so")
ISSUE_RATES = os.path.join(PKG, "issue_rates")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["dsmc_kernels.hip", "dsmc_kernels_dx1_8.hip", "dsmc_kernels_dx16.hip",
           "dsmc_kernels_dx32_f32.hip", "dsmc_kernels_dx32_f64.hip", "dsmc_api.cpp",
           "dsmc_server.cpp", "dsmc_static.cpp",
           "dsmc_pit_kalman.hip"]

# Packed-fp32 instructions are disabled for all device code (the compiler
# would otherwise form v_pk_* from plain float arithmetic).  Matrix-core
# accumulators stay in ordinary VGPRs (gfx950 has one register file): the
# default heuristic put them in AGPRs and paid a v_accvgpr_write and a
# v_accvgpr_read per accumulator element, two extra VALU slots per pair.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-Wno-unused-value",
         "-I", INCLUDE, "-I", CSRC]


# Per-source additions: the Kalman scan's in-register Gauss-Jordan inverse is
# a 32-step loop whose steps index a register array; it must unroll fully
# (else the array goes to scratch memory), past the default size limit.
EXTRA_FLAGS = {"dsmc_pit_kalman.hip": ["-mllvm", "-pragma-unroll-threshold=1000000"]}


def _compile(src: str, objdir: str) -> str:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith((".hip", ".cpp")) else []
    cmd = [HIPCC, *lang, *FLAGS, *EXTRA_FLAGS.get(src, []), "-c", os.path.join(CSRC, src),
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    # the VALU issue-rate microbenchmark behind the pair-row roofline (bench.py --issue-rates)
    cmd = [HIPCC, "-x", "hip", *[f for f in FLAGS if f != "-fPIC"],
           os.path.join(PKG, "microbench", "issue_rates.hip"), "-o", ISSUE_RATES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose:
        print(f"built {LIB} and {ISSUE_RATES}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
