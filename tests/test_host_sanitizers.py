"""The C ABI's host code under the compilers' sanitizers: the runtime sources
are compiled with AddressSanitizer + UndefinedBehaviorSanitizer on the host side
only (the device objects of the regular build, and the allocation-free entry
point's object, are linked unchanged), and a
driver (`host_sanitize_driver.cpp`) calls the host-only entry points (status
strings, shape table, finalize, record merging, the adaptive decision and their
argument checks).  Any report fails the test.  No GPU: nothing here launches a
kernel."""
import glob
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1803_07560_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1803_07560_amd", "_build")
HOST_SOURCES = ["host_pool", "runtime", "tune", "adaptive", "server", "integrand", "sampler", "resident",
                "spherical"]
# sanitizers for the host pass only (device code is never built with them)
HOST_SAN = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fno-omit-frame-pointer").split()


def test_host_entry_points_under_asan_ubsan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or shutil.which("g++") is None:
        pytest.skip("hipcc not available")
    device = sorted(glob.glob(os.path.join(BUILD, "shape_*.o")) +
                    glob.glob(os.path.join(BUILD, "is_*.o")) +
                    glob.glob(os.path.join(BUILD, "sph_*.o")) +
                    [os.path.join(BUILD, "common_kernels.o"), os.path.join(BUILD, "leaf_kernels.o"),
                     os.path.join(BUILD, "noalloc.o")])
    if not all(os.path.exists(p) for p in device) or len(device) < 3:
        pytest.skip("library not built")
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
              *HOST_SAN]
    objs = []
    for name in HOST_SOURCES:
        obj = str(tmp_path / f"{name}.o")
        r = subprocess.run([hipcc, *common, "-c", os.path.join(CSRC, f"{name}.cpp"), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    drv = str(tmp_path / "driver.o")
    r = subprocess.run([hipcc, *common, "-c", os.path.join(HERE, "host_sanitize_driver.cpp"), "-o",
                        drv], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "driver")
    r = subprocess.run([hipcc, "-o", exe, drv, *objs, *device, *HOST_SAN,
                        "-lrocprofiler-sdk-roctx", "-lpthread"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "runtime error" not in run.stderr
    assert "ERROR: AddressSanitizer" not in run.stderr
    assert "ERROR: LeakSanitizer" not in run.stderr
    assert run.stdout.strip() == "ok"
