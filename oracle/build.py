"""Build the CPU oracle (plain C, gcc) into oracle/liboracle.so.

Test infrastructure only: the device library never links or loads it.
Flags keep IEEE semantics: no fast-math, no FMA contraction (-ffp-contract=off),
so every arithmetic step of the oracle is one correctly rounded operation in
the order the source writes it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "jacobi_oracle.c")]
DEPS = SOURCES + [os.path.join(HERE, "jacobi_oracle_body.h")]


def build(verbose: bool = False) -> str:
    """Compile the oracle; always rebuilds.  Returns the library path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-o", tmp] + SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
