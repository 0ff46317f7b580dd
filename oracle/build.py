"""Build the CPU oracle shared library (test infrastructure only).

The oracle is plain C compiled without FMA contraction so that every
product and sum is rounded separately, as the rotation formula is written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rotseq_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
          "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra"]


def build(src=SRC, out=OUT, extra=()):
    """Compile ``src`` into the shared library ``out``; returns ``out``."""
    cmd = ["gcc", *CFLAGS, *extra, src, "-o", out + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(*sys.argv[1:2]))
