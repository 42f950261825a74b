"""Build libwavemodel.so and libwmbench.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2605_04178_amd.build  (or build() from Python).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libwavemodel.so")
SOURCES = ["wm_kernels.hip", "wm_tile.hip", "wm_segments.hip", "wm_planning.hip", "wm_blackwell.hip", "wm_api.cpp", "wm_tune.cpp", "wm_noalloc.hip"]
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


BENCH_OUT = os.path.join(HERE, "libwmbench.so")
BENCH_SOURCES = ["wm_microbench.hip"]


def _hipcc(out, sources, verbose, extra):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc] + FLAGS + list(extra or []) + ["-o", tmp] + [os.path.join(CSRC, s) for s in sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    return tmp


def build(verbose: bool = False, extra=None) -> str:
    """Compile libwavemodel.so (the model) and libwmbench.so (microbenchmarks
    and validation kernels)."""
    os.replace(_hipcc(OUT, SOURCES, verbose, extra), OUT)
    os.replace(_hipcc(BENCH_OUT, BENCH_SOURCES, verbose, extra), BENCH_OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
