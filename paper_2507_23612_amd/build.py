"""Build the HIP library libhcu.so for gfx950 (in-tree).

Each .hip source is compiled to an object in parallel, then linked against
rocSOLVER/rocBLAS and hipFFT.  Usage: python -m paper_2507_23612_amd.build

`--sanitize` builds lib/libhcu_san.so instead: the host code instrumented
with AddressSanitizer and UndefinedBehaviorSanitizer (every sanitizer flag
goes to the host pass only; the device code is the ordinary build).  It is
for the host-side tests (structure building, validation, error paths) and
is loaded with the sanitizer runtime preloaded (tests/test_abi_sanitized.py).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "lib")
LIB = os.path.join(OUT_DIR, "libhcu.so")
LIB_SAN = os.path.join(OUT_DIR, "libhcu_san.so")
OBJ_DIR = os.path.join(ROOT, "_build", "obj")
OBJ_DIR_SAN = os.path.join(ROOT, "_build", "obj_san")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 VALU forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]
SOURCES = ["setup.hip", "stencil.hip", "nonlocal.hip", "proj.hip", "gemm.hip", "scf_kernels.hip", "mlp.hip", "state.hip",
           "noalloc.hip", "forces.hip", "hxc.hip", "eig.hip", "api.hip"]


def _compile(src, sanitize=False):
    obj = os.path.join(OBJ_DIR_SAN if sanitize else OBJ_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *(SAN_FLAGS if sanitize else []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False, sanitize=False):
    lib = LIB_SAN if sanitize else LIB
    os.makedirs(OUT_DIR, exist_ok=True)
    os.makedirs(OBJ_DIR_SAN if sanitize else OBJ_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(s, sanitize), SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp,
           *(["-Xarch_host", "-shared-libsan", *SAN_FLAGS[:4]] if sanitize else []),
           "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
