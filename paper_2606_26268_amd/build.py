"""Build the HIP library ``libm1.so`` (gfx950) from ``csrc/``.

Each translation unit is compiled by hipcc in parallel and linked into one
shared library next to this file.  Packed-FP32 instruction selection is
switched off for device code (``-packed-fp32-ops``).
"""
from __future__ import annotations

import json
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libm1.so")
SOURCES = ["m1_api.hip", "transport.hip", "implicit.hip", "diag.hip", "mlp.hip"]
ARCH = os.environ.get("M1_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-value", "-I", os.path.join(ROOT, "include")]
# per-file code generation options: the inference kernels keep matrix-core
# accumulators in ordinary VGPRs, which the vector epilogue reads directly
FILE_FLAGS = {"implicit.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}
# the compiler's per-kernel resource remarks (registers, scratch, occupancy)
# are collected into _build/kernel_resources.json
REMARKS = ["-Rpass-analysis=kernel-resource-usage"]
_REMARK = re.compile(r"remark: +(Function Name|TotalSGPRs|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|"
                     r"Occupancy \[waves/SIMD\]|VGPRs Spill|SGPRs Spill|LDS Size \[bytes/block\]): (\S+)")
_KEYS = {"TotalSGPRs": "sgprs", "VGPRs": "vgprs", "AGPRs": "agprs", "ScratchSize [bytes/lane]": "scratch",
         "Occupancy [waves/SIMD]": "waves_per_simd", "VGPRs Spill": "vgpr_spill", "SGPRs Spill": "sgpr_spill",
         "LDS Size [bytes/block]": "lds"}


def _resources(stderr):
    """Kernel resource remarks of one compilation -> {kernel: {field: int}}."""
    out, cur = {}, None
    for line in stderr.splitlines():
        m = _REMARK.search(line)
        if not m:
            continue
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[_KEYS[key]] = int(val)
    return out


def build(verbose=False, jobs=8):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [HIPCC] + FLAGS + FILE_FLAGS.get(src, []) + REMARKS + ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        other = "\n".join(l for l in r.stderr.splitlines() if "kernel-resource-usage" not in l and l.strip()
                          and not l.lstrip().startswith(("|", "^")) and not l.lstrip()[:1].isdigit())
        if verbose and other:
            print(other, file=sys.stderr)
        return obj, _resources(r.stderr)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        done = list(ex.map(compile_one, SOURCES))
    objs = [o for o, _ in done]
    res = {}
    for _, r in done:
        res.update(r)
    with open(os.path.join(objdir, "kernel_resources.json"), "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
