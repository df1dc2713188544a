"""Compile the CPU oracle (``brandes.c``) into shared libraries next to this file.

Test infrastructure: the libraries are only loaded by the tests, the smoke check and the
benchmark's CPU-baseline leg.

* ``liboracle.so``: ``-O3`` for a generic x86-64 target, built once and carried with the tree;
* ``liboracle_native.so``: ``-O3 -march=native``, compiled on the machine that runs the CPU
  baseline, for the host-timed leg of the benchmark.

Neither build changes the arithmetic: no fast-math flag, so every floating-point sum keeps
its source order.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "brandes.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_NATIVE = os.path.join(HERE, "liboracle_native.so")

FLAGS = ["-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]


def _compile(out, extra):
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.run(["gcc"] + FLAGS + extra + ["-o", tmp, SRC], check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    return _compile(LIB, [])


def build_native() -> str:
    """The host-tuned build; always recompiled, since the host may differ from the one that
    built the tree."""
    return _compile(LIB_NATIVE, ["-march=native"])


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
