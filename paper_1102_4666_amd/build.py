"""Builds libbsde.so (HIP kernels for gfx950 + host C-ABI) in place with
hipcc, one translation unit per kernel dimension, compiled in parallel.
Run ``python -m paper_1102_4666_amd.build``."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbsde.so")
ARCH = os.environ.get("BSDE_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # no packed FP32 instructions (v_pk_*_f32) in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result", "-Wno-unused-value",
    "-fconstexpr-steps=200000000",
]


RESOURCES = os.path.join(OBJ, "resources.txt")


def _resources(text: str):
    """(kernel, VGPRs, scratch bytes per lane) from the compiler's
    kernel-resource-usage remarks."""
    out, cur = [], {}
    for ln in text.splitlines():
        if "remark:" not in ln:
            continue
        msg = ln.split("remark:", 1)[1].split(" [-Rpass")[0].strip()
        if msg.startswith("Function Name:"):
            cur = {"name": msg.split(":", 1)[1].strip()}
        elif msg.startswith("VGPRs:"):
            cur["vgprs"] = int(msg.split(":", 1)[1])
        elif msg.startswith("ScratchSize"):
            cur["scratch"] = int(msg.split(":", 1)[1])
            out.append(cur)
    return out


def _compile(src: str, verbose: bool):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [hipcc, "-x", "hip", *HIPCC_FLAGS,
           "-Rpass-analysis=kernel-resource-usage", "-c", src, "-o", obj]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    res = _resources(r.stdout + r.stderr)
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines()
            if "packed-fp32-ops" not in ln and ln.strip() and "remark" not in ln]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, "\n".join(msgs)))
    if verbose:
        print("compiled %s in %.1fs" % (os.path.basename(src), time.time() - t),
              flush=True)
        for m in msgs:
            print("  " + m)
    return obj, res


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + sorted(
        glob.glob(os.path.join(CSRC, "*.cpp")))
    # the biggest translation units first
    srcs.sort(key=lambda p: ("d10" not in p, "d5" not in p, p))
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        done = list(ex.map(lambda s: _compile(s, verbose), srcs))
    objs = [o for o, _ in done]
    with open(RESOURCES, "w") as f:
        for _, res in done:
            for k in res:
                f.write("%s vgprs=%d scratch=%d\n" % (k["name"], k["vgprs"],
                                                      k["scratch"]))
                if k["scratch"] and verbose:
                    print("WARNING: %s spills %d bytes per lane" %
                          (k["name"], k["scratch"]))
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc, "--offload-arch=" + ARCH, "-shared",
                           "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    t0 = time.time()
    print(build(verbose="-v" in sys.argv), "%.1fs" % (time.time() - t0))
