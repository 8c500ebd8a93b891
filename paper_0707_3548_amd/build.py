"""Compile the HIP library ``libtqr.so`` for gfx950 (in-tree, next to this file).

The library is split into translation units that compile in parallel: the C
entry points (tqr.hip), the batched launch (tqr_batched.hip), and one object
per supported (tile_b, inner_ib) pair (tqr_inst.hip with TQR_INST_B /
TQR_INST_IB), which holds that pair's tile kernels and persistent scheduler.

Every unit is compiled with the compiler's kernel resource-usage remarks; the
build fails when a persistent-scheduler kernel spills more scalar registers
than ``MAX_SGPR_SPILL`` or spills any vector register (a spill of scalar
values into vector-register lanes inside the scheduler kernel has produced
wrong results before, and vector spills go through scratch memory).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtqr.so")
BUILD_DIR = os.path.join(HERE, "_build")
PAIRS = [(16, 16), (32, 16), (32, 32), (64, 16), (64, 32), (64, 64), (128, 16), (128, 32), (256, 16), (256, 32)]
UNITS = [("tqr", "tqr.hip", []), ("tqr_batched", "tqr_batched.hip", []), ("tqr_noalloc", "tqr_noalloc.hip", [])] + [
    (f"tqr_b{b}_ib{ib}", "tqr_inst.hip", [f"-DTQR_INST_B={b}", f"-DTQR_INST_IB={ib}"]) for b, ib in PAIRS]
SOURCES = [os.path.join(CSRC, f) for f in ("tqr.hip", "tqr_batched.hip", "tqr_noalloc.hip", "tqr_inst.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("tqr_impl.h", "tqr_device.h", "tqr_graph.h", "tqr_narrow.h", "tqr_offsets.h")] + \
    [os.path.join(ROOT, "include", "tqr.h")]

# Scalar registers a persistent-scheduler kernel may spill (into vector
# register lanes): the instantiations spill 237 to 348 today (the scheduler's
# bookkeeping and the tile kernels share one kernel), so the limit catches
# growth, not the present state.
MAX_SGPR_SPILL = 360

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP64 matrix-core products with their accumulators in AGPRs issue at half
    # the rate of the VGPR form on gfx950 (35 vs 78 TFLOP/s measured): keep
    # every MFMA destination and accumulator in VGPRs
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]
REMARKS = ["-Rpass-analysis=kernel-resource-usage"]


def _compile(unit):
    name, src, defs = unit
    obj = os.path.join(BUILD_DIR, name + ".o")
    cmd = [HIPCC, *FLAGS, *REMARKS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    return name, obj, cmd, res


_FUNC = re.compile(r"remark: Function Name: (\S+)")
_SGPR_SPILL = re.compile(r"remark:\s+SGPRs Spill: (\d+)")
_VGPR_SPILL = re.compile(r"remark:\s+VGPRs Spill: (\d+)")


def resource_usage(text: str) -> dict:
    """Per kernel symbol: (SGPR spill count, VGPR spill count) from the
    compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in text.splitlines():
        m = _FUNC.search(line)
        if m:
            cur = m.group(1)
            out[cur] = [0, 0]
            continue
        if cur is None:
            continue
        m = _SGPR_SPILL.search(line)
        if m:
            out[cur][0] = int(m.group(1))
        m = _VGPR_SPILL.search(line)
        if m:
            out[cur][1] = int(m.group(1))
    return {k: tuple(v) for k, v in out.items()}


def check_spills(usage: dict) -> list:
    """Violations of the spill limits among the persistent-scheduler kernels."""
    bad = []
    for fn, (sgpr, vgpr) in usage.items():
        if "k_persistent" not in fn:
            continue
        if sgpr > MAX_SGPR_SPILL or vgpr > 0:
            bad.append(f"{fn}: {sgpr} SGPRs and {vgpr} VGPRs spilled (limits {MAX_SGPR_SPILL} and 0)")
    return bad


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Always recompiles every unit; returns the library path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, min(16, os.cpu_count() or 1)))
    objs, usage, failed = {}, {}, []
    with cf.ThreadPoolExecutor(max_workers=jobs) as pool:
        for name, obj, cmd, res in pool.map(_compile, UNITS):
            if verbose:
                print(" ".join(cmd), flush=True)
            if res.returncode != 0:
                failed.append(name)
                sys.stderr.write(res.stdout + "\n".join(l for l in res.stderr.splitlines() if "remark:" not in l) + "\n")
                continue
            objs[name] = obj
            usage.update(resource_usage(res.stderr))
    if failed:
        raise RuntimeError("hipcc failed to compile: " + ", ".join(failed))
    bad = check_spills(usage)
    if bad:
        raise RuntimeError("register spills beyond the limits:\n  " + "\n  ".join(bad))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *[objs[u[0]] for u in UNITS], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to link libtqr.so")
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
