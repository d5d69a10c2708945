"""Builds libtsqs.so (the HIP kernels and the C ABI of include/tsqs.h) for gfx950.

tsqs_host.hip (C ABI, workspace, queue) and one tsqs_dt.hip object per key type
are compiled in parallel, then linked into one shared library.
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtsqs.so")
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]
KEY_TYPES = 5


def _objects(tmpdir):
    jobs = [([os.path.join(CSRC, "tsqs_host.hip")], os.path.join(tmpdir, "tsqs_host.o"))]
    for dt in range(KEY_TYPES):
        jobs.append((["-DTSQS_DT=%d" % dt, os.path.join(CSRC, "tsqs_dt.hip")],
                     os.path.join(tmpdir, "tsqs_dt%d.o" % dt)))
    return jobs


def build() -> str:
    tmpdir = os.path.join(HERE, "_build")
    os.makedirs(tmpdir, exist_ok=True)
    jobs = _objects(tmpdir)

    def compile_one(job):
        args, obj = job
        subprocess.run([HIPCC] + FLAGS + ["-c"] + args + ["-o", obj], check=True)
        return obj

    workers = min(len(jobs), max(1, os.cpu_count() or 1), 16)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, jobs))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
