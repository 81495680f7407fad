"""Build the gfx950 shared library ``liblbm.so`` in-tree with hipcc.

    python -m paper_1206_0389_amd.build

Compiles every HIP source of the library for gfx950 only. Packed FP32
instructions are disabled (``-packed-fp32-ops``); the kernels are written
in scalar float/double code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = [os.path.join(HERE, "csrc", "lbm_api.hip"), os.path.join(HERE, "csrc", "lbm_refine.hip")]
HEADERS = [os.path.join(HERE, "csrc", n) for n in os.listdir(os.path.join(HERE, "csrc"))
           if n.endswith(".h")] + [os.path.join(ROOT, "include", "lbm.h")]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return ["--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include")]


def _errors(stderr: str) -> str:
    noise = "is not a recognized feature for this target"
    return "\n".join(l for l in stderr.splitlines() if noise not in l)


def build(verbose: bool = False) -> str:
    """Compiles the sources to objects concurrently, then links them."""
    import tempfile
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="lbm_build_") as tdir:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tdir, os.path.basename(src) + ".o")
            cmd = [hipcc()] + flags() + ["-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                          text=True))
            objs.append(obj)
        failed = []
        for pr in procs:
            _, err = pr.communicate()
            err = _errors(err)
            if pr.returncode != 0:
                failed.append(err)
            elif err.strip() and verbose:
                print(err, file=sys.stderr)
        if failed:
            raise RuntimeError("hipcc failed:\n" + "\n".join(failed))
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + _errors(res.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
