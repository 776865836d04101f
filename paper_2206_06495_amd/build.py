"""Compile the gfx950 HIP library ``librbffd.so`` in-tree with hipcc.

Usage: ``python paper_2206_06495_amd/build.py`` (run as a script, so that the
package, which loads the library, is not imported before the build).
Each source is compiled to an object under ``_build/`` and linked into
``paper_2206_06495_amd/librbffd.so``.  Node generation, kNN and the weight
assembly are built with -ffp-contract=off: their floating-point results are
defined operation by operation (no fused multiply-add unless written).
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librbffd.so")

SOURCES = [
    ("common.cpp", False),
    ("nodes.cpp", True),
    ("knn.hip", True),
    ("weights.hip", True),
    ("ell.hip", False),
    ("solver.hip", False),
]

ARCH = os.environ.get("RBFFD_OFFLOAD_ARCH", "gfx950")


def _hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=None):
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
              f"-I{os.path.join(ROOT, 'include')}"]
    procs = []
    objs = []
    for src, strict_fp in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        cmd = [hipcc] + common
        if src.endswith(".hip"):
            cmd += ["-x", "hip", f"--offload-arch={ARCH}",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
        if strict_fp:
            cmd += ["-ffp-contract=off"]
        cmd += ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        msg = "\n".join(f"--- {s} ---\n{t}" for s, t in failed)
        raise RuntimeError(f"HIP build failed:\n{msg}")
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print("built", LIB)
