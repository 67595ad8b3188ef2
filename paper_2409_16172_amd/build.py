"""Build the HIP library libhelmpre.so for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhelmpre.so")
SOURCES = ["hp_kernels.hip", "hp_api.cpp", "hp_spectrum.cpp"]
ARCH = os.environ.get("HP_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are kept off: the compiler would otherwise form them
# from ordinary float code.
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-munsafe-fp-atomics"]


def build(verbose: bool = False, jobs: int = 2, defines=(), out: str = LIB, objdir: str = None) -> str:
    """Compile the sources and link `out`.  `defines`: extra -D options (tuning variants)."""
    objdir = objdir or os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = ["hipcc", *HIPFLAGS, *["-D" + d for d in defines], *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
        if len(procs) >= jobs:
            p, name = procs.pop(0)
            if p.wait() != 0:
                raise RuntimeError(f"hipcc failed on {name}")
    for p, name in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {name}")
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
