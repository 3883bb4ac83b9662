"""Build the HIP library ``liblmbd.so`` for gfx950 in-tree (next to this file).

Usage: python -m paper_2407_06409_amd.build   (or call build()).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["lmbd_api.hip", "lmbd_serve.hip", "k_nbr.hip", "k_scs.hip", "k_mbd.hip", "k_gather.hip"]
LIB = os.path.join(HERE, "liblmbd.so")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread", "--offload-arch=gfx950",
    # keep hand-written float code away from the packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
