"""Builds the C oracle (test infrastructure) with gcc.

The oracle is compiled with -O2 -ffp-contract=off and without fast-math so
that every FP64 operation is one IEEE round-to-nearest operation, as written.
``mutant=k`` plants mistake k (see the BBXO_MUTANT switch in bbx_oracle.c)
for the mutation tests.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bbx_oracle.c")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD_DIR, "libbbx_oracle.so")


def build_oracle(out: str | None = None, mutant: int = 0) -> str:
    out = out or LIB
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-Werror", "-fPIC", "-shared", f"-DBBXO_MUTANT={int(mutant)}", "-o", out + ".tmp", SRC,
           "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build_oracle())
