"""The CPU oracle under the compilers' sanitizers: a driver
(`oracle_sanitize_driver.c`) calls every entry point on small inputs, threads
included, built once with AddressSanitizer + UndefinedBehaviorSanitizer and once
with ThreadSanitizer; any report fails the test.  No GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_sanitize_driver.c")]
BASE = ["-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-pthread"]


def build_and_run(tmp_path, flags, env_extra):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "driver")
    r = subprocess.run(["gcc", *BASE, *flags, "-o", exe, *SRC, "-lm"], capture_output=True,
                       text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip(f"sanitizer runtime not available: {r.stderr[:200]}")
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, **env_extra)
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    return run


def test_address_and_undefined_behaviour(tmp_path):
    run = build_and_run(tmp_path, ["-fsanitize=address,undefined",
                                   "-fno-sanitize-recover=undefined"],
                        {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0",
                         "UBSAN_OPTIONS": "print_stacktrace=1"})
    assert run.returncode == 0, run.stderr[-4000:]
    assert "runtime error" not in run.stderr
    assert "ERROR: AddressSanitizer" not in run.stderr
    assert run.stdout.strip() == "ok"


def test_threads(tmp_path):
    run = build_and_run(tmp_path, ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"})
    assert run.returncode == 0, run.stderr[-4000:]
    assert "WARNING: ThreadSanitizer" not in run.stderr
    assert run.stdout.strip() == "ok"
