"""Build libddm.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2012_05695_amd.build

Every translation unit is compiled for gfx950 only, with packed-FP32
instruction selection disabled, then linked into ``libddm.so`` next to this
file.  Object files go to ``_build/``.
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libddm.so")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

COMMON = [
    "-std=c++17", "-O3", "-fPIC",
    "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(HERE, "..", "include"),
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]

SOURCES = ["ddm_api.cpp", "mlp_api.cpp", "k_spatial.hip", "k_time.hip", "k_radial.hip", "k_fit.hip",
           "k_mlp.hip"]


def _sources():
    extra = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip") and f not in SOURCES)
    return SOURCES + extra


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    for src in _sources():
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [HIPCC, "-x", "hip", "-c", path, "-o", obj] + COMMON
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        if pr.returncode != 0:
            failed.append(src)
            sys.stderr.write(text)
        elif verbose and text.strip():
            sys.stderr.write(text)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
