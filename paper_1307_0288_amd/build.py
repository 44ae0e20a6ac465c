"""Build the gfx950 library libkpm.so in-tree with hipcc.

    python -m paper_1307_0288_amd.build      (or build() from Python)

Every call recompiles.  The library is the kernels (csrc/kpm_kernels.hip)
plus the host driver and C ABI (csrc/kpm_host.cpp, csrc/kpm_transport.cpp,
csrc/kpm_learned.cpp, include/kpm.h) and the network of the learned
reconstruction (csrc/kpm_mlp.hip).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libkpm.so")
OBJDIR = os.path.join(PKG, "_build")
SOURCES = ["kpm_kernels.hip", "kpm_host.cpp", "kpm_error.cpp", "kpm_lattice.cpp",
           "kpm_transport.cpp", "kpm_learned.cpp", "kpm_mlp.hip", "kpm_noalloc.hip",
           "kpm_march32.hip", "kpm_march_long.hip"]
# per-file device flags: the long real-part strips take the max-ILP schedule
EXTRA = {"kpm_march_long.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}
ARCH = "gfx950"


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def flags() -> list:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # packed FP32 instructions stay off: some of their forms are unreliable
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-ffp-contract=off"]


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    os.makedirs(OBJDIR, exist_ok=True)
    objs = []

    def compile_one(src):
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        # device code: the compiler's per-kernel resource report (registers,
        # spills, LDS) goes to _build/<source>.resources
        report = ["-Rpass-analysis=kernel-resource-usage"] if src.endswith(".hip") else []
        cmd = [hipcc] + flags() + EXTRA.get(src, []) + lang + report + \
            ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        if report:
            with open(os.path.join(OBJDIR, src + ".resources"), "w") as f:
                f.write(r.stderr)
        elif verbose and r.stderr.strip():
            print(r.stderr, flush=True)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def resources(src: str) -> dict:
    """Per-kernel resources of a device source from the last build: mangled
    name -> {"VGPRs", "AGPRs", "VGPRs Spill", "ScratchSize", "Occupancy",
    "LDS"}; empty when the source has not been built here."""
    import re
    path = os.path.join(OBJDIR, src + ".resources")
    if not os.path.exists(path):
        return {}
    keys = {"VGPRs": "VGPRs", "AGPRs": "AGPRs", "VGPRs Spill": "VGPRs Spill",
            "ScratchSize [bytes/lane]": "ScratchSize", "Occupancy [waves/SIMD]": "Occupancy",
            "LDS Size [bytes/block]": "LDS"}
    out, cur = {}, None
    with open(path) as f:
        for line in f:
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                cur = out.setdefault(m.group(1), {})
                continue
            m = re.search(r"remark:\s+([A-Za-z][A-Za-z /\[\]]*?): (\d+)", line)
            if m and cur is not None and m.group(1) in keys:
                cur[keys[m.group(1)]] = int(m.group(2))
    return out


if __name__ == "__main__":
    print(build(verbose=True))
