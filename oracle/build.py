"""Build the CPU oracle (``liboracle.so``) with gcc.  Test infrastructure only."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bitsort_oracle.c")
LIB_PATH = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c99", "-Wall", "-Wextra", "-Werror", "-fPIC", "-shared"]


def build_from(src: str, out: str, extra_flags=()) -> str:
    """Compile one oracle source file into a shared library at ``out``."""
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, *extra_flags, "-o", tmp, src]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_oracle() -> str:
    return build_from(SRC, LIB_PATH)


if __name__ == "__main__":
    print(build_oracle(), file=sys.stderr)
