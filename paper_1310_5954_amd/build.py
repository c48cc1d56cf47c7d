"""Builds libletkf.so (HIP kernels + C ABI runtime) for gfx950 with hipcc.

    python -m paper_1310_5954_amd.build          # or __graft_entry__.build()
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libletkf.so")
SOURCES = ["kernels.hip", "runtime.cpp", "server.cpp"]
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # keep hipcc from emitting packed FP32 VALU ops
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # MFMA sources and results in ordinary VGPRs: accumulators in AGPRs
         # would push the analysis kernel from 3 to 2 wavefronts per SIMD
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I", os.path.join(HERE, "..", "include")]


def source_hash() -> str:
    """Hash of every source and header the library is built from."""
    h = hashlib.sha256()
    # compiler flags too (without the include path, which differs per checkout)
    h.update(" ".join(f for f in FLAGS if not f.startswith(("/", "-I"))).encode())
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".hpp")))
    for f in files + ["../../include/letkf.h"]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def kernel_hash() -> str:
    """Hash of the device code alone (kernels.hip, the headers it includes and
    the compiler flags): hardware-counter summaries are keyed on it, since a
    change to the host runtime leaves the kernels' memory traffic as it was."""
    h = hashlib.sha256()
    h.update(" ".join(f for f in FLAGS if not f.startswith(("/", "-I"))).encode())
    for f in ("kernels.hip", "desc.hpp", "launch.hpp"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


RESOURCES = os.path.join(LIBDIR, "kernel_resources.json")
_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]|"
                     r"VGPRs Spill|LDS Size \[bytes/block\]): (\S+)")
_KEYS = {"VGPRs": "vgprs", "AGPRs": "agprs", "ScratchSize [bytes/lane]": "scratch_bytes",
         "Occupancy [waves/SIMD]": "waves_per_simd", "VGPRs Spill": "vgpr_spill", "LDS Size [bytes/block]": "lds_bytes"}


def _resources(stderr: str) -> dict:
    """Per-kernel register, occupancy and LDS figures from the compiler's
    resource-usage remarks (the device pass of kernels.hip)."""
    out, cur = {}, None
    for m in _REMARK.finditer(stderr):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[_KEYS[key]] = int(val)
    return out


def _compile(src: str, obj: str, build_id: str) -> None:
    remarks = ["-Rpass-analysis=kernel-resource-usage"] if src == "kernels.hip" else []
    cmd = ["hipcc", *FLAGS, *remarks, f'-DLETKF_BUILD_ID="{build_id}"', "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    if remarks:
        with open(RESOURCES + ".tmp", "w") as fh:
            json.dump({"build_id": build_id, "kernels": _resources(r.stderr)}, fh, indent=1, sort_keys=True)
        os.replace(RESOURCES + ".tmp", RESOURCES)


def build(verbose: bool = True) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    objs = [os.path.join(LIBDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    build_id = source_hash()
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(_compile, SOURCES, objs, [build_id] * len(SOURCES)))
    tmp = LIB + ".tmp"
    r = subprocess.run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    if verbose:
        print(f"built {LIB} (sources {build_id})", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
