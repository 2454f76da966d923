"""The double-precision exponential of the FP64 weights (`csrc/exp64.hpp`),
compiled for the host from the same source (its operations are IEEE fma, rint
and ldexp, exact or correctly rounded on both sides): errors below one unit in
the last place against `expl` over random arguments in [-746, 0], and the
special values (1 at 0, subnormals, 0 from -746 on and at -inf, NaN kept,
overflow to +inf).  No GPU."""
import math
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1803_07560_amd", "csrc")


def test_exp_weight_accuracy_and_special_values(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "exp_check")
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-ffp-contract=off",
                        "-I", CSRC, os.path.join(HERE, "exp_weight_check.cpp"), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120).stdout.splitlines()
    head = out[0].split()
    assert float(head[1]) < 1.0                 # faithfully rounded everywhere sampled
    assert float(head[5]) < 0.1                 # and correctly rounded for most arguments
    def parse(t):
        return math.nan if t in ("nan", "-nan") else float.fromhex(t)

    pairs = [tuple(parse(t) for t in line.split()) for line in out[1:]]
    nan_out = [y for x, y in pairs if math.isnan(x)]
    got = {x: y for x, y in pairs if not math.isnan(x)}
    assert got[0.0] == 1.0 and got[-0.0] == 1.0 and got[-1e-300] == 1.0
    assert got[-745.0] == 5e-324                # the smallest subnormal, 2^-1074
    assert got[-745.2] == 0.0                   # below 2^-1075: rounds to 0
    assert got[-746.0] == 0.0 and got[-1e308] == 0.0 and got[-math.inf] == 0.0
    assert len(nan_out) == 1 and math.isnan(nan_out[0])
    assert got[1.0] == math.e
    assert got[709.0] == pytest.approx(math.exp(709.0), rel=2e-16)
    assert got[710.0] == math.inf
