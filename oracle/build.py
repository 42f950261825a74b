"""Compile the FP64 oracle into oracle/liboracle.so (gcc, -O2, no FMA contraction).

The oracle is test infrastructure: the product library never links it.

build_variant() compiles the same sources, optionally with text replacements
or extra compiler flags, into another file: the tests use it for a build
under AddressSanitizer / UndefinedBehaviorSanitizer and for builds with a
planted mistake that a pin must catch.
"""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "wm_oracle.c"), os.path.join(HERE, "bw_oracle.c")]
OUT = os.path.join(HERE, "liboracle.so")
FLAGS = ["-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
         "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp"
    cmd = ["gcc"] + FLAGS + ["-o", tmp] + SRCS + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


def build_variant(out: str, replace=(), extra_flags=(), verbose: bool = False) -> str:
    """Build the oracle into `out`.  `replace` is a list of (file name, old,
    new) text substitutions applied to copies of the sources (each old text
    must occur exactly once); `extra_flags` are added to the gcc line."""
    work = tempfile.mkdtemp(prefix="orc_variant_")
    try:
        srcs = []
        for src in SRCS:
            text = open(src).read()
            for fname, old, new in replace:
                if fname == os.path.basename(src):
                    if text.count(old) != 1:
                        raise ValueError(f"{fname}: text to replace occurs {text.count(old)} times: {old!r}")
                    text = text.replace(old, new)
            dst = os.path.join(work, os.path.basename(src))
            with open(dst, "w") as f:
                f.write(text)
            srcs.append(dst)
        cmd = ["gcc"] + FLAGS + list(extra_flags) + ["-o", out] + srcs + ["-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    finally:
        shutil.rmtree(work, ignore_errors=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
