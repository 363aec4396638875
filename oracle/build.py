"""Build the FP64 CPU oracle (test infrastructure only).

Compiles oracle.c with gcc at -O2, IEEE semantics (no fast-math, no FMA
contraction) and OpenMP over pencils.  The result is oracle/liboracle.so.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True, src: str = SRC, lib: str = LIB) -> str:
    if not force and os.path.exists(lib) and \
            os.path.getmtime(lib) >= os.path.getmtime(src):
        return lib
    tmp = lib + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build())
