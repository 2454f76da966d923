"""The host worker pool behind the runtime's parallel loops (csrc/host_pool.*),
built with g++ on its own and run by `host_pool_check.cpp`: every chunk once,
nested loops, loops from several threads at once, exceptions from any thread
reaching the caller.  Once as built for the library (-O2) and once under
ThreadSanitizer.  No GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1803_07560_amd", "csrc")


@pytest.mark.parametrize("flags,env", [
    (["-O2"], {}),
    (["-O1", "-g", "-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"}),
], ids=["O2", "tsan"])
def test_pool_loops(tmp_path, flags, env):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "pool_check")
    r = subprocess.run(["g++", "-std=c++17", "-Wall", "-pthread", *flags, "-I", CSRC,
                        os.path.join(HERE, "host_pool_check.cpp"),
                        os.path.join(CSRC, "host_pool.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120,
                         env=dict(os.environ, **env))
    assert run.returncode == 0, run.stdout + run.stderr[-4000:]
    assert "ThreadSanitizer" not in run.stderr
    assert run.stdout.strip().endswith("ok")
    print(run.stdout.strip().splitlines()[0])
