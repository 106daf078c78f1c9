"""Builds libbloch.so (the gfx950 kernels and the C ABI of include/bloch.h) in place.

    python -m paper_2304_00337_amd.build        (or paper_2304_00337_amd.build.build())

hipcc cross-compiles for gfx950 without a GPU present.  Packed FP32 instructions are
disabled for all device code.
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SOURCES = ["csrc/stencils.hip", "csrc/dense.hip", "csrc/ritz.hip", "csrc/solver.hip",
           "csrc/abi.hip", "csrc/sched.hip", "csrc/rr.hip", "csrc/tune.hip", "csrc/coarse.hip",
           "csrc/sweep.hip", "csrc/planewave.hip",
           "csrc/noalloc.hip"]
LIB = os.path.join(PKG, "libbloch.so")
# per-source flags: the block combination and the Ritz step's products keep their MFMA
# accumulators in ordinary VGPRs (the default heuristic moves them between register files on
# every step of their loops)
EXTRA_FLAGS = {"csrc/dense.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
               "csrc/ritz.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(PKG, "csrc"),
             "-Wall", "-Wno-unused-function"]
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.basename(src).replace(".hip", ".o"))
        cmd = [hipcc(), *flags, *EXTRA_FLAGS.get(src, []), "-c", os.path.join(PKG, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src))
        objs.append(obj)
    failed = []
    for p, src in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        msg = "\n".join(f"--- {s}\n{t}" for s, t in failed)
        raise RuntimeError("HIP build failed:\n" + msg)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-ldl", "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
