"""Build the FP64 CPU oracle (test infrastructure) into oracle/liborc.so.

The oracle is plain C compiled by gcc with floating-point contraction off, so
every multiply and add rounds on its own, as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_core.c", "orc_field.c", "orc_sim.c", "orc_insert.c", "orc_spline3.c", "orc_fp32.c", "orc_insert3.c"]
LIB = os.path.join(HERE, "liborc.so")


def build(verbose=False):
    cmd = ["gcc", "-std=c11", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-D_GNU_SOURCE", "-Wall", "-Wno-unknown-pragmas",
           "-o", LIB + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_selftest(out, sanitize=True, verbose=False):
    """The stand-alone oracle driver (selftest.c) as an executable at `out`;
    with `sanitize`, under gcc's address and undefined-behaviour checks (any
    report aborts the run)."""
    flags = ["-O1", "-g", "-fno-omit-frame-pointer"]
    if sanitize:
        flags += ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    cmd = ["gcc", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-D_GNU_SOURCE", "-Wall",
           "-Wno-unknown-pragmas"] + flags + ["-o", out, os.path.join(HERE, "selftest.c")] + \
          [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
