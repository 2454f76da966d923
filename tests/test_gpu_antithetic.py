"""GPU: antithetic pairs (lattice antithetic = 1) against the oracle's.

Each sample index gives the point of its Philox words and the point of the
complemented words (the reflection through the subvolume's centre); records
sum the pair means.  Bars as for single points: FP64 records within 1e-10 of
their L1 scales, Z and C(r) within 1e-6 (FP64) and 1e-4 (FP32 form) of the
oracle's on the same pairs; launch shapes, persistent and grid kernels, plans
and graph replays agree bit for bit; the entry points without pair support
refuse it.  Then what the pairs are for: the same error bar as single points
at equal evaluations on the subvolumes of a partition."""
import json
import math

import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import assert_result_close, assert_sums_close, unshift

pytestmark = pytest.mark.gpu

F64, F32 = "fp64", "fp32"


def oracle_pairs(nx, nt, sv, seed, **kw):
    lat_o = oracle.lattice(nx, nt, antithetic=1, **kw)
    return lat_o, oracle.sums(lat_o, seed, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)


@pytest.mark.parametrize("obs", [0, 1])
@pytest.mark.parametrize("nx,nt", [(1, 1), (2, 1), (3, 2), (5, 3), (8, 2), (10, 2)])
def test_records_match_oracle(bfi, ctx, nx, nt, obs):
    d = nx * nt
    sv = workloads.random_partition(d, 3.0, 10, per_sub=1, seed=nx * 7 + nt)
    item = 64 * 256
    sv.n[:] = [2, 3, 255, 257, item - 1, item + 1, 3 * item + 17, 1000, 77, 5000]
    sv.offset[:] = [0, 5, 2**20, 3, 0, 2**33, 1, 7, 0, 123456789]
    lat_o, want = oracle_pairs(nx, nt, sv, 9, nu=0.6, observable=obs)
    lat = bfi.lattice(nx, nt, nu=0.6, observable=obs, antithetic=True)
    got = bfi.bfi_eval(ctx, lat, F64, 9, sv)
    assert np.array_equal(got[:, 0], sv.n.astype(np.float64))
    assert_sums_close(unshift(got, nx), want, nx, 1e-10)
    res_o = oracle.finalize(nx, d, sv.lo, sv.hi, want, 2)
    res = bfi.bfi_finalize(lat, sv, got)
    assert_result_close(res, res_o, 1e-6)
    assert res["n_evals"] == 2 * sv.n.sum() == res_o["n_evals"]
    got32 = bfi.bfi_eval(ctx, lat, F32, 9, sv)
    assert_result_close(bfi.bfi_finalize(lat, sv, got32), res_o, 1e-4)


@pytest.mark.parametrize("nx,nt", [(10, 2), (3, 1)])
def test_counter_boundaries(bfi, ctx, nx, nt):
    """Items whose counters cross a multiple of 2^32 (general Philox path) beside
    items that do not."""
    d = nx * nt
    nb = (d + 3) // 4
    sv = workloads.random_partition(d, 3.0, 4, per_sub=1, seed=d)
    sv.n[:] = [3000, 20_000, 5, 70_000]
    starts = []
    for k, n in zip([1, 2, 3, 5], sv.n):
        starts.append(-(-(k << 32) // nb) - int(n) // 2)
    starts[1] = 0
    sv.offset[:] = starts
    lat_o, want = oracle_pairs(nx, nt, sv, 11, nu=0.7)
    got = bfi.bfi_eval(ctx, bfi.lattice(nx, nt, nu=0.7, antithetic=True), F64, 11, sv,
                       bfi.launch(8, 64, 0))
    assert_sums_close(unshift(got, nx), want, nx, 1e-10)


@pytest.mark.parametrize("launch", [
    dict(samples_per_thread=1, block=64, persistent=0),
    dict(samples_per_thread=7, block=128, persistent=1),
    dict(samples_per_thread=64, block=256, persistent=0),
    dict(samples_per_thread=256, block=256, persistent=1),
])
def test_launch_shapes(bfi, ctx, launch):
    nx, nt = 10, 2
    sv = workloads.uniform_partition(20, 4.0, 5, per_sub=30_000)
    sv.n[3] = 17
    lat_o, want = oracle_pairs(nx, nt, sv, 1)
    got = bfi.bfi_eval(ctx, bfi.lattice(nx, nt, antithetic=True), F64, 1, sv,
                       bfi.launch(**launch))
    assert_sums_close(unshift(got, nx), want, nx, 1e-10)


def test_persistent_equals_grid_and_plans_bitwise(bfi, ctx):
    sv = workloads.random_partition(20, 4.0, 40, per_sub=30_000, seed=3)
    sv.n[::3] = 12_345
    for obs in ("anchor", "averaged"):
        lat = bfi.lattice(10, 2, nu=0.5, observable=obs, antithetic=True)
        for prec in (F64, F32):
            a = bfi.bfi_eval(ctx, lat, prec, 5, sv, bfi.launch(32, 256, 0))
            b = bfi.bfi_eval(ctx, lat, prec, 5, sv, bfi.launch(32, 256, 1))
            assert np.array_equal(a, b)
            plan = bfi.bfi_plan_create(ctx, lat, prec, sv, bfi.launch(32, 256, 1, use_graph=1))
            try:
                info = bfi.bfi_plan_info(plan)
                assert info["n_evals"] == 2 * int(sv.n.sum())
                for _ in range(3):
                    bfi.bfi_plan_run(plan, 5)
                    assert np.array_equal(bfi.bfi_plan_partials(plan, len(sv), 10), b)
            finally:
                bfi.bfi_plan_destroy(plan)


def test_integrate_counts_evaluations(bfi, ctx):
    lat = bfi.lattice(4, 2, antithetic=True)
    r = bfi.bfi_integrate(ctx, lat, F64, 1, -4.0, 4.0, 4, 1 << 20)
    assert r["n_evals"] == 1 << 20
    ref = oracle.integrate_uniform(oracle.lattice(4, 2, antithetic=1), 1, -4.0, 4.0, 4, 1 << 20)
    assert r["n_evals"] == ref["n_evals"]
    assert_result_close(r, ref, 1e-6)
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_integrate(ctx, lat, F64, 1, -4.0, 4.0, 4, 63)   # 31 pairs for 16 subvolumes
    assert e.value.name == "BFI_EINVAL"


def test_unsupported_paths_refuse_pairs(bfi, ctx):
    lat = bfi.lattice(4, 2, antithetic=True)
    sv = workloads.uniform_partition(8, 2.0, 2, per_sub=1000)
    calls = [
        lambda: bfi.bfi_eval(ctx, bfi.lattice(16, 4, antithetic=True), F64, 1,
                             workloads.uniform_partition(64, 3.0, 2, per_sub=100)),
        lambda: bfi.bfi_eval(ctx, lat, F64, 1, sv, split=True),
        lambda: bfi.bfi_integrate_adaptive(ctx, lat, F64, 1, -2.0, 2.0,
                                           bfi.adaptive_config(split_log2=2, n_min=64,
                                                               max_evals=1 << 16)),
        lambda: bfi.bfi_integrate_is(ctx, lat, F64, 1, -2.0, 2.0, 1 << 16, 0.9, 8),
        lambda: bfi.bfi_integrand_eval(ctx, bfi.integrand_burgers(lat), 1, sv),
    ]
    for call in calls:
        with pytest.raises(bfi.BfiError) as e:
            call()
        assert e.value.name == "BFI_EUNSUPPORTED"
    bad = bfi.lattice(4, 2)
    bad.antithetic = 2
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_eval(ctx, bad, F64, 1, sv)
    assert e.value.name == "BFI_EINVAL"


def test_error_bar_at_equal_evaluations(bfi, ctx):
    """10x2, nu = 1, the paper's range [-1,1]^20 in 64 subvolumes (dims 0-5
    halved): 2^19 pairs per subvolume against 2^20 single points.  The two
    weights of a pair are nearly uncorrelated on subvolumes that are not centred
    at 0, so the error bars agree; the estimates agree within them."""
    sv = workloads.uniform_partition(20, 1.0, 6, per_sub=1 << 20)
    plain = bfi.bfi_finalize(bfi.lattice(10, 2), sv,
                             bfi.bfi_eval(ctx, bfi.lattice(10, 2), F32, 1, sv))
    half = bfi.Subvolumes(sv.ids, sv.lo, sv.hi, sv.n // 2, sv.offset, 20)
    lat = bfi.lattice(10, 2, antithetic=True)
    pair = bfi.bfi_finalize(lat, half, bfi.bfi_eval(ctx, lat, F32, 2, half))
    assert pair["n_evals"] == plain["n_evals"]
    assert 0.85 < pair["Z_err"] / plain["Z_err"] < 1.15
    assert abs(pair["Z"] - plain["Z"]) < 4 * math.hypot(pair["Z_err"], plain["Z_err"])
    for r in range(10):
        assert abs(pair["C"][r] - plain["C"][r]) < 4 * math.hypot(pair["C_err"][r],
                                                                  plain["C_err"][r])


def test_full_size_sampled_in_bench_configuration(bfi, ctx):
    """The benchmark's pair launch: 10x2, nu = 1, [-4,4]^20, 2^29 pairs over 1024
    subvolumes through a resident graph plan; 3 whole subvolumes (2^19 pairs
    each) against the oracle, the FP32 form against FP64."""
    w = workloads.WORKLOADS["burgers10x2"]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, w.budget // w.n_sub // 2)
    lat = bfi.lattice(10, 2, antithetic=True)
    res = {}
    for prec in (F64, F32):
        plan = bfi.bfi_plan_create(ctx, lat, prec, sv, bfi.launch(use_graph=1))
        try:
            assert bfi.bfi_plan_info(plan)["n_evals"] == w.budget
            bfi.bfi_plan_run(plan, w.seed)
            got = bfi.bfi_plan_partials(plan, len(sv), 10)
        finally:
            bfi.bfi_plan_destroy(plan)
        res[prec] = bfi.bfi_finalize(lat, sv, got)
        if prec == F64:
            pick = np.array([0, 511, 1023])
            sub = sv.subset(pick)
            chunks = 16
            m = int(sub.n[0]) // chunks
            want = oracle.sums(oracle.lattice(10, 2, antithetic=1), w.seed,
                               np.repeat(sub.ids, chunks), np.repeat(sub.lo, chunks, axis=0),
                               np.repeat(sub.hi, chunks, axis=0), m,
                               np.tile(np.arange(chunks, dtype=np.uint64) * m, len(pick)))
            want = want.reshape(len(pick), chunks, -1).sum(1)
            assert_sums_close(unshift(got[pick], 10), want, 10, 1e-10)
    assert res[F64]["n_evals"] == w.budget
    assert_result_close(res[F32], res[F64], 1e-4)


def test_served_pairs(bfi, ctx):
    """Served pair requests: the oracle's result on the same pairs, two
    evaluations per pair, and the same records whether served alone or mixed
    with single-point requests of the same shape."""
    srv = bfi.bfi_server_create(ctx, bfi.server_config(memory_budget=1 << 30, max_requests=64,
                                                       chunks_per_step=16))
    try:
        nx, nt, B, k, budget = 4, 2, 4.0, 4, 200_004
        pair_req = bfi.request(bfi.lattice(nx, nt, nu=0.5, antithetic=True), F64, 7, B, k, budget)
        t = bfi.bfi_server_submit(srv, pair_req)
        res = bfi.bfi_server_wait(srv, t, 60.0)[0]
        ref = oracle.integrate_uniform(oracle.lattice(nx, nt, nu=0.5, antithetic=1), 7, -B, B, k,
                                       budget)
        assert res["n_evals"] == budget == ref["n_evals"]
        assert_result_close(res, ref, 1e-6)
        mix = []
        for i in range(12):
            lat = bfi.lattice(10, 2, nu=0.3 + 0.1 * i, antithetic=bool(i % 2))
            mix.append(bfi.request(lat, F32, i + 1, 2.0, 4, 1 << 18))
        tickets = [bfi.bfi_server_submit(srv, r) for r in mix]
        mixed = [bfi.bfi_server_wait(srv, t, 60.0)[0] for t in tickets]
        st = bfi.bfi_server_stats_get(srv)
        assert st["evals"] >= budget + 12 * (1 << 18)
    finally:
        bfi.bfi_server_destroy(srv)
    for i in (0, 1, 5):
        alone_srv = bfi.bfi_server_create(ctx, bfi.server_config(memory_budget=1 << 30))
        try:
            alone = bfi.bfi_server_wait(alone_srv, bfi.bfi_server_submit(alone_srv, mix[i]),
                                        60.0)[0]
        finally:
            bfi.bfi_server_destroy(alone_srv)
        assert alone["Z"] == mixed[i]["Z"] and np.array_equal(alone["C"], mixed[i]["C"]), i
        assert alone["n_evals"] == 1 << 18


def test_pairs_tuned_apart(bfi, tmp_path):
    """The pair kernel gets a tuning entry of its own (pairs = 1 in the saved
    table), which a reload restores beside the single-point entry; a tuned pair
    plan still matches the oracle.  Private contexts: the shared one keeps its
    default launches."""
    lat = bfi.lattice(4, 2, antithetic=True)
    path = str(tmp_path / "tuned.json")
    tctx = bfi.bfi_context_create(0)
    try:
        got = bfi.bfi_autotune(tctx, lat, F64, 1 << 18)
        single = bfi.bfi_autotune(tctx, bfi.lattice(4, 2), F64, 1 << 18)
        bfi.bfi_tune_save(tctx, path)
    finally:
        bfi.bfi_context_destroy(tctx)
    assert got["samples_per_thread"] >= 16 and got["block"] in (64, 128, 256, 512, 1024)
    entries = json.load(open(path))["entries"]
    mine = [e for e in entries if (e["nx"], e["nt"], e["prec"]) == (4, 2, 0)]
    assert sorted(e["pairs"] for e in mine) == [0, 1]
    pair = next(e for e in mine if e["pairs"] == 1)
    assert (pair["samples_per_thread"], pair["block"]) == (got["samples_per_thread"], got["block"])
    one = next(e for e in mine if e["pairs"] == 0)
    assert (one["samples_per_thread"], one["block"]) == (single["samples_per_thread"],
                                                          single["block"])
    ctx2 = bfi.bfi_context_create(0)
    try:
        bfi.bfi_tune_load(ctx2, path)
        sv = workloads.uniform_partition(8, 2.0, 3, per_sub=5000)
        rec = bfi.bfi_eval(ctx2, lat, F64, 4, sv)
        want = oracle.sums(oracle.lattice(4, 2, antithetic=1), 4, sv.ids, sv.lo, sv.hi, sv.n,
                           sv.offset)
        np.testing.assert_allclose(rec[:, 2:4] * np.exp(-np.array([[1, 2]]) * rec[:, 1:2]),
                                   want[:, 1:3], rtol=1e-10)
    finally:
        bfi.bfi_context_destroy(ctx2)


def test_launch_table_lookup_order(bfi, ctx, tmp_path):
    """A plan takes the table entry of its own kernel variant (pairs,
    observable); without one, the entry of its sampler with the anchored
    product; then the single-point entry.  Architecture as the context reports it,
    read back from a table the context itself saved."""
    arch_path = str(tmp_path / "arch.json")
    bfi.bfi_tune_save(ctx, arch_path)
    arch = json.load(open(arch_path))["arch"]
    entries = [  # (pairs, observable) -> samples per thread; blocks distinct too
        {"pairs": 0, "observable": 0, "samples_per_thread": 48, "block": 64},
        {"pairs": 1, "observable": 0, "samples_per_thread": 80, "block": 128},
        {"pairs": 0, "observable": 1, "samples_per_thread": 112, "block": 256},
    ]
    table = {"arch": arch, "entries": [
        dict(nx=4, nt=2, prec=0, persistent=1, evals_per_s=1.0, **e) for e in entries]}
    path = str(tmp_path / "table.json")
    json.dump(table, open(path, "w"))
    c = bfi.bfi_context_create(0)
    try:
        bfi.bfi_tune_load(c, path)
        sv = workloads.uniform_partition(8, 2.0, 2, per_sub=4096)
        want = {(False, "anchor"): (48, 64), (True, "anchor"): (80, 128),
                (False, "averaged"): (112, 256), (True, "averaged"): (80, 128)}
        for (pairs, obs), shape in want.items():
            plan = bfi.bfi_plan_create(c, bfi.lattice(4, 2, observable=obs, antithetic=pairs),
                                       F64, sv)
            try:
                info = bfi.bfi_plan_info(plan)
            finally:
                bfi.bfi_plan_destroy(plan)
            assert (info["samples_per_thread"], info["block"]) == shape, (pairs, obs)
    finally:
        bfi.bfi_context_destroy(c)
