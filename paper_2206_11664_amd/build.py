"""Build the gfx950 shared library ``libsdiag.so`` in-tree with hipcc.

Usage: ``python -m paper_2206_11664_amd.build`` (or ``build()`` from Python).
"""
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsdiag.so")
ARCH = "gfx950"

# Packed FP32 VALU forms are disabled for every HIP translation unit.
HIP_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    src = sorted(glob.glob(os.path.join(HERE, "csrc", "*.cpp")))
    src += sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    return src


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    objs = []
    for s in sources():
        o = os.path.join(out_dir, os.path.basename(s) + ".o")
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
               "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"),
               "-x", "hip", "-c", s, "-o", o] + HIP_FLAGS
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(l for l in r.stderr.splitlines()
                        if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {s}:\n{err}")
        if err.strip() and verbose:
            print(err)
        objs.append(o)
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
