"""Build libgf2ple.so (HIP, gfx950) and the input generator in-tree.

    python -m paper_1111_6549_amd.build
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgf2ple.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["api.hip", "ple_kernels.hip", "rref_kernels.hip", "prof.hip", "batch.hip", "serve.hip", "mfma.hip", "noalloc.hip", "alg3.hip"]
HEADERS = ["common.h"]

HIP_FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=" + ARCH,
    "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), res.stderr[-6000:]))
    return obj


def build_hip():
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n%s" % res.stderr[-4000:])
    os.replace(tmp, LIB)
    return LIB


def build_all():
    from . import inputs
    inputs.build(force=True)
    return build_hip()


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1111_6549_amd import build as b  # noqa: E402
    print(b.build_all())
