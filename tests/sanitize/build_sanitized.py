"""Build the library with AddressSanitizer and UndefinedBehaviorSanitizer on
its host code, and the driver that exercises it (tests/sanitize/host_exercise.cpp).

Device code is compiled as in the product build; only the host pass of each
translation unit is instrumented (every sanitizer flag follows -Xarch_host).
Outputs, in tests/sanitize/_build/: libspt_san.so and host_exercise.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
from paper_2509_00280_amd import build as product  # noqa: E402

OUT = os.path.join(HERE, "_build")
LIB = os.path.join(OUT, "libspt_san.so")
EXE = os.path.join(OUT, "host_exercise")
CLANGXX = "/opt/rocm/llvm/bin/clang++"

HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str) -> str:
    path = os.path.join(product.CSRC, src)
    obj = os.path.join(OUT, src + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [product.HIPCC, *product.COMMON, *HOST_SAN, *lang, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(_compile, product.SOURCES))
    cmd = [product.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    # the driver: host code only, built by the host compiler
    cmd = [CLANGXX, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", os.path.join(HERE, "host_exercise.cpp"), "-o", EXE,
           "-L", OUT, "-lspt_san", "-L", "/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath," + OUT, "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"driver build failed:\n{r.stdout}\n{r.stderr}")
    for o in objs:
        os.remove(o)
    if verbose:
        print(EXE, file=sys.stderr)
    return EXE


if __name__ == "__main__":
    build(verbose=True)
