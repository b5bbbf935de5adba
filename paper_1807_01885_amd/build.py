"""Compile libcoatbem.so for gfx950 with hipcc (in-tree, no JIT cache).

Every HIP source is compiled to an object in parallel, then linked into
paper_1807_01885_amd/libcoatbem.so.  Run `python -m paper_1807_01885_amd.build`.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libcoatbem.so")
BUILD_DIR = os.path.join(ROOT, "_build")

# (source, object name, extra flags): the FFT file is compiled once per
# launch-shape variant
FFT_VARIANTS = 6
SOURCES = ([("plan.cpp", "plan", []), ("fft_dispatch.cpp", "fft_dispatch", []),
            ("solver.hip", "solver", []), ("batch.cpp", "batch", []), ("net.hip", "net", []),
             ("noalloc.hip", "noalloc", []), ("layers.cpp", "layers", []),
             ("exact.cpp", "exact", [])]
           + [("fft.hip", f"fft_v{k}", [f"-DCB_FFT_VARIANT={k}"]) for k in range(FFT_VARIANTS)])
ARCH = os.environ.get("COATBEM_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep packed-FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-result",
]


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def _compile(entry):
    src, name, extra = entry
    obj = os.path.join(BUILD_DIR, name + ".o")
    cmd = [hipcc(), *COMMON, *extra]
    if src.endswith(".cpp"):
        cmd += ["-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=True):
    os.makedirs(BUILD_DIR, exist_ok=True)
    workers = min(len(SOURCES), max(1, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-lpthread", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
