"""Build liblb.so (HIP, gfx950) in-tree.

    python -m paper_2304_06437_amd.build

Compiles every csrc/*.hip translation unit with hipcc for gfx950 only (in
parallel), then links them into paper_2304_06437_amd/liblb.so.  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblb.so")
OBJ = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-signed-zeros",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = True, jobs: int | None = None) -> str:
    """Compile and link liblb.so; always recompiles."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    t = time.time()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 2)))
    objs, procs, logs = [], [], []
    pending = list(srcs)
    while pending or procs:
        while pending and len(procs) < jobs:
            src = pending.pop(0)
            obj = os.path.join(OBJ, os.path.basename(src) + ".o")
            objs.append(obj)
            cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
        src, pr = procs.pop(0)
        out, _ = pr.communicate()
        out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
        if out.strip():
            logs.append(out)
            print(out, file=sys.stderr, flush=True)
        if pr.returncode != 0:
            for _, p in procs:
                p.kill()
            raise subprocess.CalledProcessError(pr.returncode, src)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build()
