"""Compile the CPU oracle into ``oracle/liboracle.so`` with gcc.

Test infrastructure: the product library never builds or loads this.
Plain ``-O2`` without fast-math so that ``exp`` is the C library's.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")


def sources():
    return list(SRC) + sorted(
        os.path.join(HERE, f) for f in os.listdir(HERE) if f.endswith(".c") and f != "oracle.c"
    )


SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]


def build(verbose: bool = False, sanitize: bool = False, out: str = None) -> str:
    """Compile the oracle; with sanitize=True an AddressSanitizer and
    UndefinedBehaviorSanitizer build (load it with gcc's libasan preloaded)
    into `out` instead of the default library."""
    lib = out or LIB
    opt = SANITIZE_FLAGS if sanitize else ["-O2"]
    cmd = ["gcc"] + opt + ["-fPIC", "-shared", "-fopenmp", "-std=c11", "-Wall",
                           "-o", lib + ".tmp"] + sources() + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def ensure_built() -> str:
    """Build only if the library is missing or older than a source file."""
    if os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(s) <= t for s in sources()):
            return LIB
    return build()


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
