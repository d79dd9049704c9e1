"""Compile the HIP sources into the in-tree shared library ``liblqcd.so``.

Every source under ``csrc/`` is built for gfx950 only.  Object files go to
``_build/`` (git-ignored) and are rebuilt when a source or header changes;
``force=True`` rebuilds everything.  Packed FP32 instructions are disabled
(``-packed-fp32-ops``) for every device compile.

Every device compile also asks the compiler for its per-kernel resource
report (``-Rpass-analysis=kernel-resource-usage``).  The build fails if any
kernel uses private scratch memory or needs a dynamic stack: a kernel that
spills to memory runs several times slower, and scratch traffic is invisible
to the bandwidth accounting.  Register spills that stay in registers (VGPRs
parked in AGPRs, SGPRs in VGPR lanes; the report then shows spills with zero
scratch) are allowed.  The parsed report (kernel, VGPRs, AGPRs, scratch,
spills, occupancy) is written next to the objects.
"""
from __future__ import annotations

import glob
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build", "lqcd")
LIB = os.path.join(HERE, "liblqcd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Rpass-analysis=kernel-resource-usage",
]

_REMARK = re.compile(r"remark:\s+(Function Name|ScratchSize \[bytes/lane\]|VGPRs|AGPRs|"
                     r"SGPRs Spill|VGPRs Spill|Dynamic Stack|Occupancy \[waves/SIMD\]):"
                     r"\s+(\S+)")


def resource_usage(compiler_output: str):
    """Per-kernel records {name, VGPRs, AGPRs, scratch, sgpr_spill,
    vgpr_spill, dynamic_stack, occupancy} from the compiler's resource
    remarks, in the order the compiler printed them."""
    recs = []
    keys = {"ScratchSize [bytes/lane]": "scratch", "SGPRs Spill": "sgpr_spill",
            "VGPRs Spill": "vgpr_spill", "Dynamic Stack": "dynamic_stack",
            "Occupancy [waves/SIMD]": "occupancy", "VGPRs": "VGPRs", "AGPRs": "AGPRs"}
    for key, val in _REMARK.findall(compiler_output):
        if key == "Function Name":
            recs.append({"name": val})
        elif recs:
            recs[-1][keys[key]] = val
    return recs


def resource_violations(recs):
    """Kernels that use scratch memory (spills to memory included) or need a
    dynamic stack."""
    return [r for r in recs
            if r.get("scratch", "0") != "0" or r.get("dynamic_stack", "False") != "False"]


def _headers():
    return glob.glob(os.path.join(CSRC, "*.h")) + [
        os.path.join(os.path.dirname(HERE), "include", "lqcd.h")]


def _compile(src: str, obj: str) -> None:
    cmd = [HIPCC, *DEVICE_FLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed for {os.path.basename(src)}")
    recs = resource_usage(res.stderr)
    with open(obj + ".resources.txt", "w") as f:
        for r in recs:
            f.write(" ".join(f"{k}={v}" for k, v in r.items()) + "\n")
    bad = resource_violations(recs)
    if bad:
        os.remove(obj)
        lines = "\n".join(" ".join(f"{k}={v}" for k, v in r.items()) for r in bad)
        raise RuntimeError(f"{os.path.basename(src)}: kernels with scratch memory or a dynamic "
                           f"stack:\n{lines}")


def build(force: bool = False, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    sources = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    newest_header = max(os.path.getmtime(h) for h in _headers())
    jobs = []
    objs = []
    for src in sources:
        obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
        objs.append(obj)
        stale = (force or not os.path.exists(obj)
                 or os.path.getmtime(obj) < max(os.path.getmtime(src), newest_header))
        if stale:
            jobs.append((src, obj))
    if jobs:
        if verbose:
            print(f"[lqcd build] compiling {len(jobs)} source(s) for gfx950", flush=True)
        with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
            list(ex.map(lambda j: _compile(*j), jobs))
    if jobs or force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv)
    print(LIB)
