"""Build libsquint.so for gfx950 with hipcc (sources compiled in parallel).

Usage: python -m paper_2602_21203_amd.build   (or build() from Python)
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsquint.so")
OBJ = os.path.join(HERE, "_build")

SOURCES = [
    "kernels/rng.hip", "kernels/squint.hip", "kernels/gemm.hip", "kernels/rowops.hip", "kernels/adam.hip", "kernels/serve.hip", "kernels/encoder.hip", "kernels/env.hip",
    "layout.cpp", "twins.cpp", "ops.cpp", "abi.cpp", "noalloc.hip", "agent.cpp", "server.cpp", "ring.cpp", "env.cpp",
]
ARCH = os.environ.get("SQ_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-fvisibility=hidden",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-function"]


def hipcc():
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


def _compile(src):
    obj = os.path.join(OBJ, src.replace("/", "_") + ".o")
    cmd = [hipcc(), *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{err}")
    return obj, err


def build(verbose=False, out=None, extra=()):
    """Compile every source and link libsquint.so (or `out`); `extra` adds
    compiler flags (e.g. -D tuning macros for experiments)."""
    os.makedirs(OBJ, exist_ok=True)
    FLAGS.extend(extra)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        results = list(ex.map(_compile, SOURCES))
    for _, err in results:
        if verbose and err.strip():
            print(err)
    objs = [o for o, _ in results]
    target = out or OUT
    tmp = target + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fvisibility=hidden", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n" + r.stdout + r.stderr)
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
