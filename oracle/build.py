"""Build the FP64 CPU oracle (test infrastructure only).

Compiles oracle.c with gcc at -O2, IEEE semantics (no fast-math, no FMA
contraction) and OpenMP over pencils.  The result is oracle/liboracle.so.
build(sanitize=True) adds AddressSanitizer and UndefinedBehaviorSanitizer
(every report fatal) for a CPU-only test of the oracle's memory accesses and
arithmetic; that library needs the ASan runtime preloaded into the process
that loads it (asan_runtime()).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-std=c11", "-Wall", "-Wextra"]
SANITIZE = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=all"]


def build(force: bool = True, src: str = SRC, lib: str = LIB, sanitize: bool = False) -> str:
    if not force and os.path.exists(lib) and \
            os.path.getmtime(lib) >= os.path.getmtime(src):
        return lib
    tmp = lib + ".tmp"
    flags = CFLAGS + (SANITIZE if sanitize else [])
    cmd = ["gcc", *flags, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def asan_runtime() -> str:
    """Path of gcc's AddressSanitizer runtime (to LD_PRELOAD)."""
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], check=True,
                         capture_output=True, text=True).stdout.strip()
    return os.path.realpath(out)


if __name__ == "__main__":
    print(build())
