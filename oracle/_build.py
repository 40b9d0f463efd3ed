"""Compile the oracle's C core into ``oracle/liboracle.so`` with gcc.

Plain -O2: no fast-math, so IEEE division and square root round correctly.
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(_HERE, "oracle.c")]


def library_path() -> str:
    return os.path.join(_HERE, "liboracle.so")


def stale() -> bool:
    out = library_path()
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    return any(os.path.getmtime(s) > t for s in SOURCES)


def build() -> str:
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-o", tmp] + SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
