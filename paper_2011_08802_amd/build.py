"""Build the mvpf libraries for gfx950 with hipcc (in-tree).

Each ``csrc/*.hip`` translation unit is compiled to an object under
``_build/`` in parallel and linked into one shared library per number of
martensite variants N (a compile-time constant of the kernels):
``paper_2011_08802_amd/libmvpf.so`` (N = 6, the CuAlNi workloads) and
``paper_2011_08802_amd/libmvpf_n12.so`` (N = 12, 15 unknowns per node).
Always recompiles (the caller decides when to build).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MVPF_ARCH", "gfx950")
NVARS = (6, 12)


def lib_path(nvar: int) -> str:
    return os.path.join(HERE, "libmvpf.so" if nvar == 6 else f"libmvpf_n{nvar}.so")


LIB = lib_path(6)

CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-result",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(job) -> str:
    src, nvar = job
    obj = os.path.join(BUILD, f"n{nvar}", os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, f"-DMVPF_NVAR={nvar}", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} (N = {nvar}):\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if warn:
        sys.stderr.write(warn + "\n")
    return obj


def build(jobs: int | None = None, nvars=NVARS) -> str:
    srcs = sources()
    work = [(src, n) for n in nvars for src in srcs]
    for n in nvars:
        os.makedirs(os.path.join(BUILD, f"n{n}"), exist_ok=True)
    jobs = jobs or min(len(work), os.cpu_count() or 4, 16)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, work))
    for n in nvars:
        lib = lib_path(n)
        tmp = lib + ".tmp"
        mine = [o for (src, m), o in zip(work, objs) if m == n]
        cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *mine]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed (N = {n}):\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build())
