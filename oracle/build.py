"""Compiles the oracle (plain C) into ``oracle/liboracle_b64.so`` with gcc.

Test infrastructure only: the codec library never links or loads this.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "b64_oracle.c")
LIB = os.path.join(HERE, "liboracle_b64.so")
CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread"]


def build(extra_flags=(), out=LIB, src=SRC):
    """Compile the oracle; returns the path of the shared library."""
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra_flags, src, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
