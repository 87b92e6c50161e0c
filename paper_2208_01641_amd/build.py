"""Builds the HIP library liblic.so in-tree for gfx950.

HIP sources go through hipcc (device code for gfx950 only, packed-FP32 ops
disabled); the host-only runtime, entropy coder and C ABI are compiled by
g++ (no FMA contraction, so the FP64 table construction is plain IEEE) and
everything is linked by hipcc.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblic.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIP_SOURCES = ["conv_kernels.hip", "distill_kernels.hip", "context_kernels.hip"]
CPP_SOURCES = ["entropy.cpp", "packing.cpp", "model.cpp", "pipeline.cpp", "server.cpp", "api.cpp", "distill.cpp"]

HIPCC = [os.path.join(ROCM, "bin", "hipcc"), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
CXX = ["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
       "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include")]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    return out


def _stale(obj: str, src: str) -> bool:
    """An object is stale if it is missing or older than its source or any
    header the sources include (csrc/*.h, include/*.h)."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    hdrs = [os.path.join(SRC, h) for h in os.listdir(SRC) if h.endswith(".h")]
    inc = os.path.join(os.path.dirname(HERE), "include")
    hdrs += [os.path.join(inc, h) for h in os.listdir(inc) if h.endswith(".h")]
    return any(os.path.getmtime(p) >= t for p in [src] + hdrs)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compiles every source (incremental=True: only stale objects) and links."""
    os.makedirs(OUT, exist_ok=True)
    jobs = []
    objs = []
    for f in HIP_SOURCES:
        o = os.path.join(OUT, f + ".o")
        if not incremental or _stale(o, os.path.join(SRC, f)):
            jobs.append(HIPCC + ["-c", os.path.join(SRC, f), "-o", o])
        objs.append(o)
    for f in CPP_SOURCES:
        o = os.path.join(OUT, f + ".o")
        if not incremental or _stale(o, os.path.join(SRC, f)):
            jobs.append(CXX + ["-c", os.path.join(SRC, f), "-o", o])
        objs.append(o)
    with ThreadPoolExecutor(max_workers=max(1, min(8, len(jobs)))) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run(HIPCC + ["-shared", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
