"""Build the gfx950 shared library ``librtsdf.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC_DIR = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librtsdf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed fp32 VALU instructions: the kernels are written for one fp32 operation per lane and instruction
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]

# The translation units and their extra flags.  The JFA's device code holds no NaNs (its keys are non-negative
# denormals or a large finite value, its coarse SDF finite), and compiled without NaN semantics a minimum of two
# keys is one v_min_f64 instead of a v_max_f64 that quiets signalling NaNs plus the v_min_f64.  Host code keeps
# NaN semantics (its argument checks test for NaN).
UNITS = [
    ("rtsdf_lib.hip", []),
    ("jfa.hip", ["-Xarch_device", "-fno-honor-nans"]),
]


def sources() -> list[str]:
    return sorted(os.path.join(SRC_DIR, f) for f in os.listdir(SRC_DIR)
                  if f.endswith((".hip", ".hpp")))


def _run(cmd: list[str], verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build librtsdf.so")


def build(verbose: bool = False) -> str:
    """Compile every translation unit (in parallel) and link them into librtsdf.so."""
    objs, procs = [], []
    for src, extra in UNITS:
        obj = os.path.join(SRC_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-c", os.path.join(SRC_DIR, src),
               "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = False
    for cmd, pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            sys.stderr.write(" ".join(cmd) + "\n" + out)
            failed = True
    if failed:
        raise RuntimeError("hipcc failed to build librtsdf.so")
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    for o in objs:
        os.remove(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
