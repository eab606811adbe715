"""Build the HIP library libigafem.so in-tree with hipcc for gfx950.

Usage: python -m paper_2207_00280_amd.build   (or build() from Python)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libigafem.so")
SOURCES = ["host.cpp", "batch.cpp", "tables.hip", "element.hip", "rows_tile.hip", "rows_geo.hip", "adjoint.hip", "apply.hip", "euler.hip", "geometry.hip", "assemble.hip", "wq.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-I" + os.path.join(os.path.dirname(HERE), "include")]


def build(verbose=False, jobs=8):
    os.makedirs(OBJ, exist_ok=True)
    procs = []
    objs = []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(OBJ, s + ".o")
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
        if s.endswith(".cpp"):
            cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if out.returncode:
        sys.stderr.write(out.stdout.decode())
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    name, p = item
    out, _ = p.communicate()
    text = out.decode()
    if p.returncode:
        sys.stderr.write(text)
        raise RuntimeError("hipcc failed on " + name)
    lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if lines:
        sys.stderr.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
