"""Build libpfmp.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_1609_02652_amd.build  (or build() from Python).
Every call recompiles; objects go to a temporary directory, the shared library
to paper_1609_02652_amd/libpfmp.so.
"""
import concurrent.futures
import glob
import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpfmp.so")
ARCH = os.environ.get("PFMP_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # no packed FP32 instructions (v_pk_*_f32) in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _compile(src, obj):
    cmd = [HIPCC, "-c", src, "-o", obj] + FLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (os.path.basename(src), r.stderr[-6000:]))
    return obj


def build(verbose=False, jobs=None):
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    tmp = tempfile.mkdtemp(prefix="pfmp_build_")
    try:
        objs = [os.path.join(tmp, os.path.basename(s) + ".o") for s in srcs]
        jobs = jobs or min(8, os.cpu_count() or 4)
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            list(ex.map(_compile, srcs, objs))
        out = LIB + ".tmp"
        cmd = [HIPCC, "-shared", "-o", out] + objs + ["--offload-arch=" + ARCH, "-fPIC"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stderr[-4000:])
        os.replace(out, LIB)
        if verbose:
            print("built", LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
