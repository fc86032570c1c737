"""Compile libobg.so (all HIP sources) for gfx950 with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libobg.so")
SOURCES = ["kernels.hip", "api.hip", "probe.hip", "batch.hip", "serve.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _jobs() -> int:
    for key in ("MAX_JOBS", "OMP_NUM_THREADS"):
        try:
            return max(1, int(os.environ[key]))
        except (KeyError, ValueError):
            pass
    return max(1, min(len(SOURCES), os.cpu_count() or 1))


def build(verbose: bool = False, extra=()) -> str:
    """Compile every source (in parallel, one hipcc per file) and link."""
    objs = [os.path.join(CSRC, src.replace(".hip", ".o")) for src in SOURCES]

    def compile_one(i):
        cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-c", os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(min(_jobs(), len(SOURCES))) as ex:
        list(ex.map(compile_one, range(len(SOURCES))))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
