"""Build libsf.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

Usage: python -m paper_1711_02473_amd.build_lib  (or build() from Python).
Every source is compiled on every call (the build check compiles from
scratch); objects go to _build/ next to this file, the library to
paper_1711_02473_amd/libsf.so.
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsf.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          "-I" + os.path.join(os.path.dirname(HERE), "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip"] + COMMON + DEVICE + ["-c", src, "-o", obj]
    else:
        cmd = [HIPCC] + COMMON + ["-D__HIP_PLATFORM_AMD__", "-c", src, "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    return src, obj, r.returncode, r.stdout, cmd


def build(jobs=None, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(16, max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    objs = []
    failed = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, obj, rc, out, cmd in ex.map(_compile, srcs):
            if rc != 0:
                failed.append((src, out, cmd))
            elif verbose and out.strip():
                print(out)
            objs.append(obj)
    if failed:
        for src, out, cmd in failed:
            sys.stderr.write("=== build failed: %s\n%s\n%s\n" % (src, " ".join(cmd), out))
        raise RuntimeError("hipcc failed for %d source(s)" % len(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout)
    os.replace(tmp, LIB)
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
