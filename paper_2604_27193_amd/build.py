"""Build the HIP library ``libaeb.so`` for gfx950 in-tree.

Every source under ``csrc/`` is compiled (in parallel) with
``-ffp-contract=off`` (no implicit multiply-add fusion: the kernels' fused
operations are the explicit ``fma`` calls) and packed FP32 instructions
disabled.
"""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libaeb.so")
ARCH = os.environ.get("AEB_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{INCLUDE}", f"-I{CSRC}", "-pthread",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(force: bool = True, extra=()) -> str:
    """Compile the library (one object per source, in parallel, then one
    link); returns the path of the shared object."""
    srcs = sources()
    deps = srcs + glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(INCLUDE, "aeb.h")]
    if not force and os.path.exists(LIB):
        if os.path.getmtime(LIB) >= max(os.path.getmtime(p) for p in deps):
            return LIB
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cflags = [f for f in FLAGS if f not in ("-shared",)]
    procs, objs = [], []
    for src in srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        procs.append((src, subprocess.Popen(["hipcc", *cflags, *extra, "-c", "-o", obj, src])))
    bad = [src for src, p in procs if p.wait() != 0]
    if bad:
        raise subprocess.CalledProcessError(1, "hipcc", output=f"failed: {bad}")
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-pthread", *extra,
                    "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
