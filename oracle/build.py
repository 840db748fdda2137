"""Build the CPU oracle library (test infrastructure only).

The oracle is plain C compiled with gcc, no fast-math and no FMA contraction, so every
expression rounds exactly as written in the source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["fas_oracle.c"]
DEPS = ["fas_oracle.c", "fas_oracle_body.h"]
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra"]


def build(force=True):
    """Compile liboracle.so in place; returns its path."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(os.path.join(HERE, d)) for d in DEPS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + CFLAGS + ["-o", tmp] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
