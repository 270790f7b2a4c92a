"""Host-code sanitizer builds (AddressSanitizer + UndefinedBehaviorSanitizer).

Builds the library with its host code (octree planner, C ABI, launch code)
instrumented -- device code is compiled as usual -- and the CPU oracle, into
``paper_2112_15198_amd/_build/sanitized/``.  CPU only; the sanitized library
is never loaded on a GPU.  Run the CPU tests against them with the
sanitizer runtimes preloaded, as printed by ``main``.
"""
from __future__ import annotations

import os
import subprocess

from . import build as B

OUT = os.path.join(B.HERE, "_build", "sanitized")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def build_library() -> str:
    os.makedirs(OUT, exist_ok=True)
    objs = []
    for src in B.SOURCES:
        obj = os.path.join(OUT, src + ".o")
        flags = [f for f in B.HIPCC_FLAGS if f != "-O3"] + ["-O1", "-g"] + HOST_SAN
        subprocess.run([B.hipcc()] + flags + ["-I", os.path.join(B.ROOT, "include"), "-c",
                                              os.path.join(B.CSRC, src), "-o", obj], check=True)
        objs.append(obj)
    lib = os.path.join(OUT, "libifgf_sanitized.so")
    subprocess.run([B.hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib] + objs,
                   check=True)
    return lib


def build_oracle() -> str:
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "libifgf_oracle_sanitized.so")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", "-o", lib,
                    os.path.join(B.ROOT, "oracle", "ifgf_oracle.cpp")], check=True)
    return lib


def main():
    lib = build_library()
    orc = build_oracle()
    rt = subprocess.run([B.hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    print(f"library: {lib}\noracle:  {orc}")
    print("library CPU tests (clang runtime):\n"
          f"  ASAN_OPTIONS=detect_leaks=0 LD_PRELOAD={rt} IFGF_LIB_PATH={lib} "
          "python -m pytest tests/test_library_cpu.py -m 'not gpu'")
    print("oracle CPU tests (gcc runtimes):\n"
          "  ASAN_OPTIONS=detect_leaks=0 LD_PRELOAD=$(g++ -print-file-name=libasan.so):"
          f"$(g++ -print-file-name=libubsan.so) IFGF_ORACLE_PATH={orc} "
          "python -m pytest tests/test_oracle_direct.py tests/test_oracle_ifgf.py")


if __name__ == "__main__":
    main()
