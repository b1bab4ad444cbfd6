"""Build step for the FP64 reference (test infrastructure only).

Compiles ``aeb_oracle.c`` into ``liborc.so`` next to this file with gcc,
``-O2 -ffp-contract=off -fno-fast-math`` so that no multiply-add is fused
except where the source calls ``fma`` explicitly, and ``-fno-builtin`` so
that each libm call is the function the source names (gcc would otherwise
merge sin and cos of one argument into one sincos call, whose last bit
differs from sin's and cos's for some arguments).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "aeb_oracle.c")
HDR = os.path.join(HERE, "aeb_oracle.h")
LIB = os.path.join(HERE, "liborc.so")

CFLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fno-builtin", "-fPIC", "-shared",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force: bool = True) -> str:
    """Compile the reference library; returns the path of the shared object."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(SRC), os.path.getmtime(HDR))
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
