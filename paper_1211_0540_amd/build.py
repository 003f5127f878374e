"""Build libbz.so (HIP, gfx950) in-tree.

Every HIP source is compiled with packed FP32 instructions disabled
(-packed-fp32-ops); hipcc's host pass warns that it does not know the
feature, which is harmless.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbz.so")
SOURCES = ["bz_runtime.hip", "bz_dft.hip", "bz_misc.hip", "bz_conv.hip", "bz_transport.hip", "bz_mlp.hip", "bz_surrogate.hip"]
ARCH = os.environ.get("BZ_OFFLOAD_ARCH", "gfx950")


def hipcc_flags():
    return ["-O3", "-std=c++20", f"--offload-arch={ARCH}", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", os.path.join(HERE, "..", "include")]


def build(verbose: bool = False, jobs: int = 4) -> str:
    objs = []
    procs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src.replace(".hip", ".o"))
        cmd = ["hipcc", *hipcc_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
        while len([p for p, _ in procs if p.poll() is None]) >= jobs:
            procs[[p.poll() is None for p, _ in procs].index(True)][0].wait()
    for p, src in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {src}")
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
