"""GPU: single integrands on the paper's integrand protocol and the paper's own
subdivision policy (section 3; criteria ranges of section 4).

  * The N-sphere integrand equals the oracle's on the same Philox points, and
    reproduces the paper's Listing 2: half the volume of the 3-ball within 4
    sigma and the printed error bar 4.355e-4 for 1e7 samples over [-1,1]^2.
  * The subdivision driver on Listing 1's problem (3-D integrand, [-1,1]^3)
    agrees with the closed form pi^2/4 and with the paper's printed result.
  * The lattice integrands equal V sum/n of the oracle's sums.
  * The command-line adapters speak the paper's line protocol and flags."""
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_listings.json")))


def half_ball(n):
    return math.pi ** (n / 2) / math.gamma(n / 2 + 1) / 2


def box(dim, lo, hi, n, sub_id=1):
    return workloads.SubvolumeList(np.array([sub_id], np.uint64), np.full((1, dim), lo),
                                   np.full((1, dim), hi), np.array([n], np.uint64),
                                   np.array([0], np.uint64))


@pytest.mark.parametrize("dim", [1, 2, 3, 5, 16])
def test_nsphere_matches_oracle(bfi, ctx, dim):
    n = 200_003
    res, err, _ = bfi.bfi_integrand_eval(ctx, bfi.integrand_nsphere(dim), 1, box(dim, -1.0, 1.0,
                                                                                  n, 7))
    want = oracle.nsphere(dim, 1, -1.0, 1.0, n, sub_id=7)
    assert res[0] == pytest.approx(want["result"], rel=1e-12)
    assert err[0] == pytest.approx(want["abserr"], rel=1e-9)


def test_listing2_on_gpu(bfi, ctx):
    g = GOLDEN["listing2"]
    res, err, dim = bfi.bfi_integrand_eval(ctx, bfi.integrand_nsphere(g["dim"]), 1,
                                           box(g["dim"], g["lo"], g["hi"], g["samples"]))
    assert abs(res[0] - half_ball(3)) < 4 * err[0]
    assert err[0] == pytest.approx(g["abserr"], rel=3e-3)
    assert dim[0] in (0, 1)


def test_split_suggestion_follows_the_variation(bfi, ctx):
    """f varies strongly along x near the sphere's edge and hardly along y near
    y = 0: the suggested split is x (and y once the box is transposed)."""
    f = bfi.integrand_nsphere(2)
    sv = workloads.SubvolumeList(np.array([1, 2], np.uint64),
                                 np.array([[0.5, -0.05], [-0.05, 0.5]]),
                                 np.array([[0.99, 0.05], [0.05, 0.99]]),
                                 np.array([100_000, 100_000], np.uint64), np.zeros(2, np.uint64))
    _, _, dim = bfi.bfi_integrand_eval(ctx, f, 3, sv)
    assert list(dim) == [0, 1]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-4)])
def test_lattice_integrands_match_oracle(bfi, ctx, prec, tol):
    nx, nt = 4, 2
    sv = workloads.uniform_partition(8, 2.0, 2, per_sub=5000)
    sums = oracle.sums(oracle.lattice(nx, nt, nu=0.8), 4, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    V = np.prod(sv.hi - sv.lo, axis=1)
    lat = bfi.lattice(nx, nt, nu=0.8)
    z, ez, _ = bfi.bfi_integrand_eval(ctx, bfi.integrand_burgers(lat, prec), 4, sv)
    np.testing.assert_allclose(z, V * sums[:, 1] / 5000, rtol=tol)
    sd = np.sqrt((sums[:, 2] - sums[:, 1] ** 2 / 5000) / 4999)
    np.testing.assert_allclose(ez, V * sd / np.sqrt(5000), rtol=max(tol, 1e-8))
    n2, _, _ = bfi.bfi_integrand_eval(ctx, bfi.integrand_burgers(lat, prec, 2), 4, sv)
    scale = V * np.sqrt(sums[:, 3 + nx + 2] * 5000) / 5000
    assert np.all(np.abs(n2 - V * sums[:, 3 + 2] / 5000) <= tol * scale)


def test_hdi_listing1(bfi, ctx):
    g = GOLDEN["listing1"]
    # 4096 + 8192 samples per subvolume and a 1 % criterion force subdivision
    cfg = bfi.hdi_config(n_initial=4096, sample_factor=2.0, rel_diff=1.01, max_depth=12,
                         max_evals=1 << 32)
    out = bfi.bfi_integrate_hdi(ctx, bfi.integrand_nsphere(g["dim"]), 1, g["lo"], g["hi"], cfg)
    assert out["status"] == "BFI_OK"
    assert out["generations"] >= 2 and out["accepted"] >= 2
    assert abs(out["result"] - half_ball(4)) < 4 * out["abserr"]
    # consistent with the paper's own printed result and error bar
    assert abs(out["result"] - g["result"]) < 4 * math.hypot(out["abserr"], g["abserr"])


def test_hdi_criteria(bfi, ctx):
    f = bfi.integrand_nsphere(2)
    # a generous relative criterion accepts the initial partition at once
    easy = bfi.bfi_integrate_hdi(ctx, f, 1, -1.0, 1.0, bfi.hdi_config(
        n_initial=4096, rel_diff=10.0, split_log2=3, max_evals=1 << 30))
    assert easy["generations"] == 1 and easy["accepted"] == 8 and easy["unconverged"] == 0
    assert easy["evals"] == 8 * (4096 + 8192)
    # criterion 3 (both results small) accepts everything too
    small = bfi.bfi_integrate_hdi(ctx, f, 1, -1.0, 1.0, bfi.hdi_config(
        n_initial=4096, rel_diff=0.0, max_abs=10.0, split_log2=2, max_evals=1 << 30))
    assert small["generations"] == 1 and small["accepted"] == 4
    # no criterion: every subvolume splits down to max_depth
    deep = bfi.bfi_integrate_hdi(ctx, f, 1, -1.0, 1.0, bfi.hdi_config(
        n_initial=4096, rel_diff=0.0, split_log2=1, max_depth=3, max_evals=1 << 30))
    assert deep["accepted"] == 16 and deep["unconverged"] == 16 and deep["depth"] == 3
    assert abs(deep["result"] - half_ball(3)) < 5 * deep["abserr"]
    # a budget that cannot pay for the children stops the refinement
    poor = bfi.bfi_integrate_hdi(ctx, f, 1, -1.0, 1.0, bfi.hdi_config(
        n_initial=4096, rel_diff=0.0, split_log2=1, max_depth=10, max_evals=2 * 12288 + 100))
    assert poor["status"] == "BFI_EBUDGET" and poor["accepted"] == 2


def test_hdi_burgers_ratio(bfi, ctx):
    """The paper's run: 10x2 lattice, integration range [-1, 1]; C(5) = N(5)/Z
    from two subdivision runs agrees with a uniform 2^28-point estimate."""
    lat = bfi.lattice(10, 2)
    cfg = bfi.hdi_config(n_initial=1 << 16, sample_factor=2.0, rel_diff=1.085, max_depth=4,
                         split_log2=4, max_evals=1 << 27)
    z = bfi.bfi_integrate_hdi(ctx, bfi.integrand_burgers(lat), 11, -1.0, 1.0, cfg)
    n5 = bfi.bfi_integrate_hdi(ctx, bfi.integrand_burgers(lat, "fp64", 5), 12, -1.0, 1.0, cfg)
    c5 = n5["result"] / z["result"]
    e5 = abs(c5) * math.hypot(n5["abserr"] / n5["result"], z["abserr"] / z["result"])
    ref = bfi.bfi_integrate(ctx, lat, "fp64", 13, -1.0, 1.0, 10, 1 << 28)
    assert abs(c5 - ref["C"][5]) < 4 * math.hypot(e5, ref["C_err"][5])


def run_module(mod, args, stdin=""):
    env = dict(os.environ, PYTHONPATH=ROOT)
    return subprocess.run([sys.executable, "-m", mod, *args], input=stdin, capture_output=True,
                          text=True, timeout=240, env=env, cwd=ROOT)


def test_cli_line_protocol(bfi):
    out = run_module("paper_1803_07560_amd.integrand",
                     ["--integrand", "integrands/N-sphere", "--dimensions", "2"],
                     "1e6 -1 1 -1 1\n100000 0 1 0 1\n")
    assert out.returncode == 0, out.stderr
    lines = out.stdout.strip().splitlines()
    assert len(lines) == 2
    r, e, j = lines[0].split()
    assert abs(float(r) - half_ball(3)) < 4 * float(e) and int(j) in (0, 1)
    r2, e2, _ = lines[1].split()
    assert abs(float(r2) - half_ball(3) / 4) < 4 * float(e2)


def test_cli_hdintegrator(bfi):
    out = run_module("paper_1803_07560_amd.hdintegrator",
                     ["--integrand", "integrands/N-sphere", "--dimensions", "3",
                      "--min-extent", "-1", "--max-extent", "1", "--samples", "65536",
                      "--max-depth", "8"])
    assert out.returncode == 0, out.stderr
    r, e = (float(v) for v in out.stdout.split())
    assert abs(r - half_ball(4)) < 4 * e
