"""Build librogs.so (hand-written HIP for gfx950) in-tree with hipcc, and the
serving runtime's host-sanitizer test driver."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librogs.so")
OBJ = os.path.join(ROOT, "_build")
SOURCES = ["api.hip", "project.hip", "sort.hip", "render.hip", "loss_adam.hip", "autotune.hip",
           "serve.hip", "grid.hip", "bev.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden",
    # no packed-FP32 instructions anywhere in the library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]

# The serving runtime's test driver: host code under AddressSanitizer and
# UndefinedBehaviorSanitizer, device code as in the library.
SAN_DRIVER = os.path.join(ROOT, "tests", "serve_sanitize_driver.cpp")
SAN_EXE = os.path.join(ROOT, "tests", "_bin", "serve_sanitize")
SAN_FLAGS = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
             "-Xarch_host -fno-sanitize-recover=all -Xarch_host -fno-omit-frame-pointer").split()


def _jobs() -> int:
    return max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))


def _compile_all(flags, sub: str, verbose: bool):
    """Compiles every library source to an object under _build/<sub> in
    parallel; returns the object paths."""
    os.makedirs(os.path.join(OBJ, sub), exist_ok=True)

    def one(src):
        obj = os.path.join(OBJ, sub, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(_jobs()) as ex:
        return list(ex.map(one, SOURCES))


def build(verbose: bool = False) -> str:
    """Compile every HIP source into librogs.so (always recompiles)."""
    objs = _compile_all(FLAGS, "lib", verbose)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_serve_sanitizer(verbose: bool = False) -> str:
    """The serving-runtime test driver (tests/serve_sanitize_driver.cpp)
    linked with the library sources, host code built with ASan and UBSan."""
    flags = ["--offload-arch=gfx950", "-O1", "-gline-tables-only", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SAN_FLAGS
    objs = _compile_all(flags, "san", verbose)
    drv = os.path.join(OBJ, "san", "serve_sanitize_driver.o")
    cmds = [[HIPCC] + flags + ["-c", SAN_DRIVER, "-o", drv]]
    os.makedirs(os.path.dirname(SAN_EXE), exist_ok=True)
    tmp = SAN_EXE + ".tmp"
    cmds.append([HIPCC, "--offload-arch=gfx950"] + SAN_FLAGS + [drv] + objs +
                ["-lpthread", "-o", tmp])
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_EXE)
    return SAN_EXE


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
    if "--sanitizer" in sys.argv:
        print(build_serve_sanitizer(verbose="-v" in sys.argv))
