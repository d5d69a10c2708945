"""Builds libtsqs.so (the HIP kernels and the C ABI of include/tsqs.h) for gfx950."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtsqs.so")
SOURCES = [os.path.join(HERE, "csrc", "tsqs_host.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def build() -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC] + FLAGS + SOURCES + ["-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
