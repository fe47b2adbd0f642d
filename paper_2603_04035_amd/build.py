"""Build the gfx950 shared library libknn.so from csrc/*.hip with hipcc.

Flags: -O3, C++17, position independent, code for gfx950 only, and packed
FP32 instructions disabled in device code (v_pk_* FP32 forms are not
emitted).  The library is written next to this file so that it travels with
the source tree.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libknn.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False, jobs: int = 4) -> str:
    objs = []
    cmds = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in sources():
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        objs.append(obj)
        cmds.append([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                     "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                     "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj])
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


def _wait(p):
    _, err = p.communicate()
    lines = [l for l in (err or "").splitlines()
             if "packed-fp32-ops' is not a recognized feature" not in l]
    if lines:
        sys.stderr.write("\n".join(lines) + "\n")
    if p.returncode != 0:
        raise RuntimeError("hipcc failed: " + " ".join(p.args))


if __name__ == "__main__":
    print(build(verbose=True))
