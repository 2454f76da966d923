"""Build ``libbfi.so`` (HIP kernels for gfx950 + host runtime + C ABI) in-tree.

Two objects per lattice shape (``shape_kernels.hip`` and the sampler's
``is_kernels.hip``, compiled with -DBFI_NX/-DBFI_NT for every shape listed in
``csrc/internal.h``), one for the shape-independent kernels, and the host
runtime; linked into ``paper_1803_07560_amd/libbfi.so``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbfi.so")
MICROBENCH = os.path.join(HERE, "microbench", "issue_rates")
ARCH = os.environ.get("BFI_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# packed FP32 instructions stay disabled in device code; hipcc's host pass warns
# that it does not know the feature, which is harmless
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"]
HOST_SOURCES = ["host_pool.cpp", "runtime.cpp", "tune.cpp", "adaptive.cpp", "server.cpp", "integrand.cpp",
                "sampler.cpp", "resident.cpp", "spherical.cpp"]


def shapes() -> list[tuple[int, int]]:
    txt = open(os.path.join(CSRC, "internal.h")).read()
    m = re.search(r"#define BFI_SHAPES\(X\)(.*?)\n\n", txt, re.S)
    if not m:
        raise RuntimeError("BFI_SHAPES not found in internal.h")
    return [(int(a), int(b)) for a, b in re.findall(r"X\((\d+),\s*(\d+)\)", m.group(1))]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stderr}")
    return r


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    jobs = jobs or min(8, os.cpu_count() or 1)
    tasks = []
    for nx, nt in shapes():
        obj = os.path.join(BUILD, f"shape_{nx}x{nt}.o")
        tasks.append([cc, *COMMON, *DEVICE, f"-DBFI_NX={nx}", f"-DBFI_NT={nt}", "-c",
                      os.path.join(CSRC, "shape_kernels.hip"), "-o", obj])
        tasks.append([cc, *COMMON, *DEVICE, f"-DBFI_NX={nx}", f"-DBFI_NT={nt}", "-c",
                      os.path.join(CSRC, "is_kernels.hip"), "-o",
                      os.path.join(BUILD, f"is_{nx}x{nt}.o")])
        tasks.append([cc, *COMMON, *DEVICE, f"-DBFI_NX={nx}", f"-DBFI_NT={nt}", "-c",
                      os.path.join(CSRC, "sph_kernels.hip"), "-o",
                      os.path.join(BUILD, f"sph_{nx}x{nt}.o")])
    for src in ("common_kernels.hip", "leaf_kernels.hip", "noalloc.hip"):
        tasks.append([cc, *COMMON, *DEVICE, "-c", os.path.join(CSRC, src), "-o",
                      os.path.join(BUILD, src.replace(".hip", ".o"))])
    for src in HOST_SOURCES:
        tasks.append([cc, *COMMON, "-c", os.path.join(CSRC, src), "-o",
                      os.path.join(BUILD, src.replace(".cpp", ".o"))])
    # the issue-rate microbenchmark (a standalone program, not part of the library)
    bench_task = [cc, "-O3", "-std=c++17", *DEVICE, os.path.join(HERE, "microbench",
                                                                 "issue_rates.hip"),
                  "-o", MICROBENCH + ".tmp"]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), tasks + [bench_task]))
    os.replace(MICROBENCH + ".tmp", MICROBENCH)
    objs = [t[t.index("-o") + 1] for t in tasks]
    _run([cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", LIB + ".tmp", *objs,
          "-lrocprofiler-sdk-roctx", "-lpthread"], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
