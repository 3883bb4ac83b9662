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


def build_host_sanitized(out_dir: str, verbose: bool = False) -> str:
    """A copy of the library whose host code carries AddressSanitizer and
    UndefinedBehaviorSanitizer (device code as in the release build), for checking
    the host side of the C ABI without a GPU.  Returns the path of the library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "liblmbd_hostsan.so")
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"]
    for opt in ("-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer",
                "-fno-sanitize-recover=undefined"):
        flags += ["-Xarch_host", opt]
    cmd = [hipcc, *flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=not verbose)
    return out


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
