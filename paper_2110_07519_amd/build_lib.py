"""Compile libmessi.so (HIP, gfx950) in-tree with hipcc.

FP contraction is off everywhere: the summary pass must round every FP32
step exactly once to give the words the index is defined by; where a kernel
wants a fused multiply-add it calls it explicitly.  FP32 division and
square root are correctly rounded (the z-normalisation's standard deviation
is a sqrtf whose result must equal IEEE's), which the flag pins rather than
leaving it to the compiler's default.  Packed FP32 ops are disabled (the
kernels use scalar FP32/FP64 arithmetic only).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmessi.so")
SOURCES = ["build.hip", "query.hip", "api.cpp"]
FLAGS = ["-std=c++17", "-O3", "--offload-arch=gfx950", "-ffp-contract=off",
         "-fhip-fp32-correctly-rounded-divide-sqrt", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]


def build(hipcc: str = "hipcc", verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        objs.append(obj)
        cmd = [hipcc] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stderr=subprocess.PIPE, stdout=subprocess.PIPE))
    for src, pr in zip(SOURCES, procs):
        out, err = pr.communicate()
        msg = "\n".join(l for l in err.decode().splitlines() if "packed-fp32-ops" not in l)
        if pr.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{msg}")
        if verbose and msg.strip():
            print(msg, file=sys.stderr)
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
