"""Build the plain C oracle into ``oracle/liboracle.so`` with gcc.

The oracle is test infrastructure: it checks the GPU library and shares no
code with it.  ``python -m oracle.build`` (or ``build()``) always recompiles.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "iwpp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    """Compile iwpp_oracle.c (C11, -O2, single-threaded) and return the path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-fPIC", "-shared", SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
