"""Build libmknn.so (the HIP library behind include/mknn.h) for gfx950.

    python -m paper_1412_6170_amd.build

Flags that matter for the result contract:
  -ffp-contract=off                 no fused multiply-add anywhere
  -fno-gpu-flush-denormals-to-zero  fp32 denormals kept
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                    no packed fp32 instructions
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", f) for f in ("index.hip", "query.hip", "query_wave.hip",
                                              "query_group.hip", "capi.hip")]
OUT = os.path.join(HERE, "libmknn.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]


def build(verbose=False, extra=()):
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + list(extra) + ["-o", tmp] + SRC
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
