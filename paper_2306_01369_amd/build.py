"""Build libgg.so (HIP, gfx950) in place next to this file."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = [os.path.join(HERE, "csrc", "gg.hip")]
HEADERS = [os.path.join(HERE, "csrc", "kernels.hip.h"), os.path.join(ROOT, "include", "gg.h")]

# Packed FP32 instructions are disabled in device code (-packed-fp32-ops).
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-I" + os.path.join(ROOT, "include")]


def lib_path():
    return os.path.join(HERE, "libgg.so")


def build(verbose=False):
    out = lib_path()
    tmp = out + ".tmp"
    cmd = [HIPCC] + FLAGS + SOURCES + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
