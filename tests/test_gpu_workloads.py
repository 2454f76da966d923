"""Whole-workload parity: the benchmark's workloads at full size, in the launch
configuration the benchmark times (resident graph plan, the committed tuned
launch table), against the FP64 oracle on the same points.

* 10x2 (nu = 1, [-4,4]^20, 2^30 points over 1024 subvolumes): the oracle runs
  all 2^30 points.  FP64 and shifted FP64: every record field within 1e-10 of
  its L1 scale, Z (log Z) within 1e-6, C(r) within 1e-6 of its L1 scale
  sum_s V_s/n_s sum |p_r w| / Z, C_err within 1e-6.  FP32 form: Z and C(r)
  within its stated 1e-4 of the oracle (not of the GPU's FP64 result).
* 16x4 (nu = 0.5, [-3,3]^64, 2^34 points over 4096 subvolumes): the full
  launch as timed, with three whole subvolumes (2^22 points each) against the
  oracle; and the stratified subset of the first 2^14 samples of every one of
  the 4096 subvolumes (2^26 points) in the same launch shape, whole against the
  oracle, both forms.
The oracle uses the host's CPU share (at most 16 threads)."""
import os

import numpy as np
import pytest

import oracle
import workloads
from parity_util import assert_records_close, assert_result_close, c_scale, move_shift

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNED = os.path.join(ROOT, "paper_1803_07560_amd", "tuned_gfx950.json")


def _threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def bench_ctx(bfi):
    c = bfi.bfi_context_create(0)
    bfi.bfi_tune_load(c, TUNED)
    yield c
    bfi.bfi_context_destroy(c)


def _plan_records(bfi, ctx, lat, prec, sv, seed):
    print(f"workload: plan {prec} {len(sv)} subvolumes {int(sv.n.sum())} samples", flush=True)
    plan = bfi.bfi_plan_create(ctx, lat, prec, sv, bfi.launch(use_graph=1))
    try:
        info = bfi.bfi_plan_info(plan)
        bfi.bfi_plan_run(plan, seed)
        got = bfi.bfi_plan_partials(plan, len(sv), lat.nx)
    finally:
        bfi.bfi_plan_destroy(plan)
    return got, info


def _split_l1(rec, nx):
    L = oracle.sums_len(nx)
    return rec[:, :L], rec[:, L:]


@pytest.fixture(scope="module")
def oracle_10x2():
    w = workloads.WORKLOADS["burgers10x2"]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, w.budget // w.n_sub)
    print(f"workload: oracle over all {w.budget} points of {w.name} on {_threads()} threads",
          flush=True)
    rec = oracle.sums_l1(oracle.lattice(10, 2), w.seed, sv.ids, sv.lo, sv.hi, sv.n, sv.offset,
                         nthreads=_threads())
    plain, l1 = _split_l1(rec, 10)
    res = oracle.finalize(10, 20, sv.lo, sv.hi, plain)
    return w, sv, plain, l1, res


@pytest.mark.parametrize("prec", ["fp64", "fp64s"])
def test_config_10x2_whole_workload_fp64(bfi, bench_ctx, oracle_10x2, prec):
    w, sv, plain, l1, res_o = oracle_10x2
    lat = bfi.lattice(10, 2)
    got, info = _plan_records(bfi, bench_ctx, lat, prec, sv, w.seed)
    assert info["n_evals"] == 2**30 and got[:, 0].sum() == 2**30
    assert info["use_graph"] == 1
    worst = assert_records_close(move_shift(got, 10, 0.0), plain, l1, 10, 1e-10)
    res_g = bfi.bfi_finalize(lat, sv, got)
    err = assert_result_close(res_g, res_o, c_scale(sv.lo, sv.hi, plain, l1), 1e-6)
    print(f"workload: 10x2 {prec} records {worst:.2e} of L1, result {err}", flush=True)


def test_config_10x2_whole_workload_fp32_form(bfi, bench_ctx, oracle_10x2):
    w, sv, plain, l1, res_o = oracle_10x2
    lat = bfi.lattice(10, 2)
    got, info = _plan_records(bfi, bench_ctx, lat, "fp32", sv, w.seed)
    assert info["n_evals"] == 2**30 and got[:, 0].sum() == 2**30
    res_g = bfi.bfi_finalize(lat, sv, got)
    scale = c_scale(sv.lo, sv.hi, plain, l1)
    err = assert_result_close(res_g, res_o, scale, 1e-4)
    print(f"workload: 10x2 fp32 form vs oracle {err}", flush=True)


def _subset_check(bfi, ctx, nx, nt, params, sv, seed, tol64=1e-6, tol32=1e-4):
    lat = bfi.lattice(nx, nt, **params)
    print(f"workload: oracle over {int(sv.n.sum())} points on {_threads()} threads", flush=True)
    rec = oracle.sums_l1(oracle.lattice(nx, nt, **params), seed, sv.ids, sv.lo, sv.hi, sv.n,
                         sv.offset, nthreads=_threads())
    plain, l1 = _split_l1(rec, nx)
    res_o = oracle.finalize(nx, nx * nt, sv.lo, sv.hi, plain)
    scale = c_scale(sv.lo, sv.hi, plain, l1)
    for prec, tol in (("fp64", tol64), ("fp32", tol32)):
        got, _ = _plan_records(bfi, ctx, lat, prec, sv, seed)
        if prec == "fp64":
            assert_records_close(move_shift(got, nx, 0.0), plain, l1, nx, 1e-10)
        assert_result_close(bfi.bfi_finalize(lat, sv, got), res_o, scale, tol)


def test_config_16x4_stratified_subset(bfi, bench_ctx):
    """The first 2^14 samples of each of the 4096 subvolumes of the 16x4
    workload (2^26 points), whole, against the oracle."""
    w = workloads.WORKLOADS["burgers16x4"]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, 1 << 14)
    _subset_check(bfi, bench_ctx, 16, 4, dict(nu=0.5), sv, w.seed)


def test_config_16x4_full_launch_whole_subvolumes(bfi, bench_ctx):
    """The full 2^34-point launch as timed; subvolumes 0, 2047 and 4095 (2^22
    points each) against the oracle in both forms, field by field in FP64 and
    as a three-subvolume estimate in the FP32 form."""
    w = workloads.WORKLOADS["burgers16x4"]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, w.budget // w.n_sub)
    lat = bfi.lattice(16, 4, nu=0.5)
    pick = np.array([0, 2047, 4095])
    sub = sv.subset(pick)
    rec = oracle.sums_l1(oracle.lattice(16, 4, nu=0.5), w.seed, sub.ids, sub.lo, sub.hi, sub.n,
                         sub.offset, nthreads=_threads())
    plain, l1 = _split_l1(rec, 16)
    res_o = oracle.finalize(16, 64, sub.lo, sub.hi, plain)
    scale = c_scale(sub.lo, sub.hi, plain, l1)
    for prec, tol in (("fp64", 1e-6), ("fp32", 1e-4)):
        got, info = _plan_records(bfi, bench_ctx, lat, prec, sv, w.seed)
        assert info["n_evals"] == 2**34 and got[:, 0].sum() == 2**34
        if prec == "fp64":
            assert_records_close(move_shift(got[pick], 16, 0.0), plain, l1, 16, 1e-10)
        assert_result_close(bfi.bfi_finalize(lat, sub, got[pick]), res_o, scale, tol)


def test_config_4x2_whole_workload(bfi, bench_ctx):
    """4x2 (nu = D = 1, [-4,4]^8, 2^20 points over 16 subvolumes) in the tuned
    launch, whole against the oracle."""
    w = workloads.WORKLOADS["burgers4x2"]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, w.budget // w.n_sub)
    _subset_check(bfi, bench_ctx, 4, 2, {}, sv, w.seed)
