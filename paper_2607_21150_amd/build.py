"""Build libpfmf.so (HIP, gfx950) in-tree with hipcc: the C-ABI unit and one unit per FP64
apply mode, compiled in parallel, then linked."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
UNITS = ["pfmf.hip", "pf_op_res.hip", "pf_op_jac.hip", "pf_op_adj.hip"]
OBJ_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpfmf.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-I" + os.path.join(ROOT, "include"),
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _run(cmd):
    return subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = [os.path.join(OBJ_DIR, os.path.splitext(u)[0] + ".o") for u in UNITS]
    cmds = [[hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, u), "-o", o] for u, o in zip(UNITS, objs)]
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        results = list(ex.map(_run, cmds))
    for cmd, res in zip(cmds, results):
        if res.returncode != 0:
            sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed on {os.path.basename(cmd[-3])}")
        if verbose:
            sys.stderr.write(res.stderr)
    tmp = LIB + ".tmp"
    res = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking libpfmf.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
