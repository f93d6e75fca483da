"""Compile the su2fft HIP library for gfx950 into the package directory."""
from __future__ import annotations

import json
import os
import re
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsu2fft.so")
# per-kernel register, scratch and occupancy figures the compiler reported for
# the library last built (a build product, next to the library)
RESOURCES = os.path.join(HERE, "kernel_resources.json")
# su2fft_kernels.hip is the one translation unit of the transform kernels: it
# includes su2fft_ring.hip, su2fft_ring_fast.hip, su2fft_beta.hip and
# su2fft_beta_bf16.hip and adds the work-list kernels of mixed plans
SOURCES = ["su2fft_host.hip", "su2fft_kernels.hip", "su2fft_table.hip", "su2fft_calib.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: the compiler must not form v_pk_* FP32 ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    # the compiler's per-kernel resource report (registers, scratch, occupancy)
    "-Rpass-analysis=kernel-resource-usage",
]

_FIELDS = {"VGPRs": "vgprs", "AGPRs": "agprs", "TotalSGPRs": "sgprs", "ScratchSize [bytes/lane]": "scratch_bytes",
           "Occupancy [waves/SIMD]": "occupancy", "LDS Size [bytes/block]": "static_lds_bytes",
           "VGPRs Spill": "vgpr_spill", "SGPRs Spill": "sgpr_spill"}


def _demangle(names):
    tool = shutil.which("llvm-cxxfilt") or shutil.which("c++filt") or "/opt/rocm/llvm/bin/llvm-cxxfilt"
    if not os.path.exists(tool):
        return {n: n for n in names}
    res = subprocess.run([tool], input="\n".join(names), capture_output=True, text=True)
    out = res.stdout.splitlines()
    return dict(zip(names, out)) if len(out) == len(names) else {n: n for n in names}


def parse_resource_report(text: str) -> dict:
    """{kernel: {vgprs, agprs, sgprs, scratch_bytes, occupancy, static_lds_bytes}}
    from the compiler's kernel-resource-usage remarks."""
    kernels, cur = {}, None
    for line in text.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = kernels.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+(.+?): (\S+) \[-Rpass-analysis", line)
        if m and cur is not None and m.group(1) in _FIELDS:
            v = m.group(2)
            cur[_FIELDS[m.group(1)]] = int(v) if v.isdigit() else v
    names = _demangle(sorted(kernels))
    return {names[k]: v for k, v in kernels.items()}


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    with open(RESOURCES, "w") as fh:
        json.dump(parse_resource_report(res.stderr), fh, indent=1, sort_keys=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
