"""Build ``libhmc.so`` (the HIP library behind include/hmc.h) in-tree.

``hipcc --offload-arch=gfx950`` cross-compiles without a GPU.  All HIP code is
built with packed FP32 instructions disabled.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libhmc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def headers():
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    return hs + [os.path.join(ROOT, "include", "hmc.h")]


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer (the device code is
# built as usual); load such a build with clang's ASan runtime preloaded.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build(verbose: bool = False, jobs: int = 8, sanitize_host: bool = False, out: str = None) -> str:
    """Compile every HIP source for gfx950 and link libhmc.so (or `out`)."""
    lib = out or LIB
    objdir = os.path.dirname(lib) if out else CSRC
    objs = []
    procs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src)[:-4] + ".o")
        cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-c",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", obj, src]
        if sanitize_host:
            cmd[1:1] = HOST_SANITIZE
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
        if len(procs) >= jobs:
            p, s = procs.pop(0)
            if p.wait() != 0:
                raise RuntimeError(f"hipcc failed on {s}")
    for p, s in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {s}")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    for o in objs:
        os.remove(o)
    return lib


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in sources() + headers())


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
