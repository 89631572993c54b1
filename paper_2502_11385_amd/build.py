"""Build libqsv.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2502_11385_amd.build   (or __graft_entry__.build())
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build", "qsv")
LIB = os.path.join(HERE, "libqsv.so")

SOURCES = ["api.cpp", "planner.cpp", "batch.cpp", "server.cpp", "cut.cpp",
           "k_outputs.hip", "k_permute.hip",
           "k_gate.hip", "k_cut.hip", "k_stream.hip",
           "k_tile.hip", "k_reduce.hip", "k_fused.hip", "k_batch.hip"]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          f"-I{INCLUDE}", f"-I{CSRC}", "-Wall", "-Wno-unused-function"]
# Packed FP32 instructions stay disabled on this target.
DEVICE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Keep switch arms over register indices separate: merging them turns
# constant register-array indices into dynamic ones, which forces the
# register-resident tile into scratch memory.
NO_SINK = ["-mllvm", "-simplifycfg-sink-common=false"]
# The register-tile kernels (tile passes, batch phases) also leave uniform
# control flow unstructured: structurizing the op loop's uniform switch
# (over an op's class and target register) into flow blocks with partly
# undefined phis made the register allocator copy every amplitude register
# after every op (32 moves per 128 FMAs).  Only these files, which the
# parity suite covers op class by op class: the cut reconstruction kernels
# gave wrong results with it.
UNSTRUCTURED = ["-mllvm", "-structurizecfg-skip-uniform-regions=true"]
TILE_SOURCES = ("k_tile.hip", "k_batch.hip")


# The compiler's per-kernel resource report (registers, scratch, spills,
# occupancy) of each device source, kept beside its object file.
RESOURCES = ["-Rpass-analysis=kernel-resource-usage"]
_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|"
                     r"ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]|"
                     r"VGPRs Spill|SGPRs Spill|LDS Size \[bytes/block\]): "
                     r"(\S+)")


def resource_table(stderr: str) -> str:
    """One line per kernel: name, then key=value fields of the report."""
    rows, cur = [], None
    for m in _REMARK.finditer(stderr):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = [val]
            rows.append(cur)
        elif cur is not None:
            cur.append(f"{key.split(' [')[0].replace(' ', '_')}={val}")
    return "".join(" ".join(r) + "\n" for r in rows)


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + DEVICE
    if src.endswith(".hip"):
        cmd += ["-x", "hip"] + NO_SINK + RESOURCES
        if src in TILE_SOURCES:
            cmd += UNSTRUCTURED
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if src.endswith(".hip"):
        with open(os.path.splitext(obj)[0] + ".resources.txt", "w") as f:
            f.write(resource_table(r.stderr))
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
        objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
