"""Builds the HIP library libqsim355.so in-tree for gfx950.

    python -m paper_2604_12256_amd.build

Every source is compiled by hipcc (HIP kernels and host C++ alike) into
_build/ at the repository root, then linked into
paper_2604_12256_amd/libqsim355.so.  Packed FP32 instructions are disabled for
device code.

The HIP sources are compiled with the compiler's per-kernel resource report
(VGPRs, AGPRs, SGPRs, spills, private-segment size, occupancy).  The parsed
table is written next to the library (libqsim355.resources.json), and the
build fails when any kernel needs private (scratch) memory or a dynamic
stack: a kernel whose registers spill to scratch runs far slower, and a large
private segment per lane can make the queue refuse the dispatch at run time
(HSA_STATUS_ERROR_OUT_OF_RESOURCES) instead of failing here.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libqsim355.so")
RESOURCES = os.path.join(PKG, "libqsim355.resources.json")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["api.cpp", "gates.cpp", "plan.cpp", "kernels_basic.hip", "kernel_small.hip", "kernel_stage.hip",
           "kernel_mfma.hip", "kernels_measure.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"),
          "-I", CSRC]
DEVICE = ["-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast"]


REPORT = ["-Rpass-analysis=kernel-resource-usage"]
_REMARK = re.compile(r"remark:\s+(.+?):\s+(\S+)\s+\[-Rpass-analysis=kernel-resource-usage\]")


def parse_resource_report(text: str) -> dict:
    """Per-function table from the compiler's kernel-resource-usage remarks:
    {function: {"VGPRs": 240, "ScratchSize [bytes/lane]": 0, ...}}."""
    table, cur = {}, None
    for m in _REMARK.finditer(text):
        key, val = m.group(1).strip(), m.group(2)
        if key == "Function Name":
            cur = table.setdefault(val, {})
            continue
        if cur is None:
            continue
        if val in ("True", "False"):
            cur[key] = val == "True"
        else:
            try:
                cur[key] = int(val)
            except ValueError:
                cur[key] = val
    return table


def scratch_offenders(table: dict) -> list:
    """Functions that need private memory per lane or a dynamic stack."""
    return sorted(f for f, r in table.items()
                  if r.get("ScratchSize [bytes/lane]", 0) > 0 or r.get("Dynamic Stack", False))


def _compile(src: str):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    hip = src.endswith(".hip")
    cmd = [HIPCC] + COMMON + DEVICE + (REPORT if hip else []) + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj, (parse_resource_report(r.stderr) if hip else {})


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        done = list(ex.map(_compile, srcs))
    objs = [o for o, _ in done]
    table = {}
    for _, t in done:
        table.update(t)
    with open(RESOURCES + ".tmp", "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(RESOURCES + ".tmp", RESOURCES)
    bad = scratch_offenders(table)
    if bad:
        raise RuntimeError("kernels need scratch memory (registers spill or a dynamic stack): " +
                           ", ".join(f"{f} ({table[f].get('ScratchSize [bytes/lane]')} B/lane)" for f in bad))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + [
        "-Wl,-rpath,/opt/rocm/lib", "-L/opt/rocm/lib", "-lamdhip64", "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
