"""Build step for the CPU oracle (plain g++, OpenMP).  Test infrastructure."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    """The in-tree oracle library, or IFGF_ORACLE_PATH (a sanitized build)."""
    return os.environ.get("IFGF_ORACLE_PATH") or os.path.join(HERE, "libifgf_oracle.so")


def build() -> str:
    src = os.path.join(HERE, "ifgf_oracle.cpp")
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
           "-o", tmp, src]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
