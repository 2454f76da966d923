"""GPU: the translation-averaged observable (p_r averaged over every anchor of
the lattice) against the oracle's, through the C ABI.

Same bars as the anchored parity tests: sums within 1e-10 of their L1 scale,
Z and C(r) within 1e-6 (FP64) / 1e-4 (FP32 form); plus what the averaged
product adds: C(r) and C(nx - r) bit-identical, and a smaller error bar than the
anchored product on the same points with a consistent value."""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_parity import assert_result_close, assert_sums_close, unshift

pytestmark = pytest.mark.gpu

F64, F32 = "fp64", "fp32"
AVG = "averaged"


def both(bfi, ctx, nx, nt, sv, seed, prec=F64, launch=None, params=None, split=False):
    params = params or {}
    want = oracle.sums(oracle.lattice(nx, nt, observable=1, **params), seed, sv.ids, sv.lo, sv.hi,
                       sv.n, sv.offset)
    got = bfi.bfi_eval(ctx, bfi.lattice(nx, nt, observable=AVG, **params), prec, seed, sv, launch,
                       split=split)
    return want, got


def test_4x2_full_workload(bfi, ctx):
    w = workloads.WORKLOADS["burgers4x2"]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, w.budget // w.n_sub)
    want, got = both(bfi, ctx, 4, 2, sv, w.seed)
    assert_sums_close(unshift(got, 4), want, 4, 1e-10)
    lat = bfi.lattice(4, 2, observable=AVG)
    res_o = oracle.finalize(4, 8, sv.lo, sv.hi, want)
    res_g = bfi.bfi_finalize(lat, sv, got)
    assert_result_close(res_g, res_o, 1e-6)
    np.testing.assert_allclose(res_g["C_err"], res_o["C_err"], rtol=1e-6)
    assert res_g["C"][1] == res_g["C"][3]
    res_i = bfi.bfi_integrate(ctx, lat, F64, w.seed, -w.box, w.box, w.split_log2, w.budget)
    assert res_i["Z"] == res_g["Z"] and np.array_equal(res_i["C"], res_g["C"])


@pytest.mark.parametrize("nx,nt", [(1, 2), (2, 1), (2, 2), (3, 2), (5, 3), (8, 2), (10, 2)])
def test_ragged_partition_odd_and_even_nx(bfi, ctx, nx, nt):
    """nx = 1 and 2 (the pair at r = nx/2 doubled), odd and even nx; uneven
    counts around the work-item size and nonzero offsets."""
    d = nx * nt
    sv = workloads.random_partition(d, 4.0, 8, per_sub=1, seed=nx * 10 + nt)
    item = 64 * 256
    sv.n[:] = [2, 3, 257, item - 1, item + 1, 3 * item + 17, 1000, 5000]
    sv.offset[:] = [0, 5, 2**20, 3, 2**33, 7, 0, 123456789]
    want, got = both(bfi, ctx, nx, nt, sv, 7, params=dict(nu=0.6))
    assert_sums_close(unshift(got, nx), want, nx, 1e-10)
    for r in range(1, nx):
        assert np.array_equal(got[:, 4 + r], got[:, 4 + nx - r])


@pytest.mark.parametrize("nx,nt,box", [(4, 2, 4.0), (10, 2, 4.0), (8, 2, 4.0), (16, 4, 3.0)])
def test_fp32_form(bfi, ctx, nx, nt, box):
    d = nx * nt
    sv = workloads.uniform_partition(d, box, 4, per_sub=20_000)
    want, got = both(bfi, ctx, nx, nt, sv, 1, prec=F32)
    res_o = oracle.finalize(nx, d, sv.lo, sv.hi, want)
    assert_result_close(bfi.bfi_finalize(bfi.lattice(nx, nt, observable=AVG), sv, got), res_o,
                        1e-4)


@pytest.mark.parametrize("launch", [dict(samples_per_thread=1, block=64, persistent=0),
                                    dict(samples_per_thread=64, block=256, persistent=1),
                                    dict(samples_per_thread=16, block=128, persistent=1),
                                    dict(samples_per_thread=16, block=512, persistent=1),
                                    dict(samples_per_thread=7, block=1024, persistent=0)])
def test_launch_shapes(bfi, ctx, launch):
    sv = workloads.uniform_partition(20, 4.0, 4, per_sub=30_000)
    sv.n[3] = 17
    want, got = both(bfi, ctx, 10, 2, sv, 2, launch=bfi.launch(**launch))
    assert_sums_close(unshift(got, 10), want, 10, 1e-10)


def test_persistent_equals_grid_bitwise(bfi, ctx):
    sv = workloads.random_partition(20, 4.0, 24, per_sub=30_000, seed=4)
    lat = bfi.lattice(10, 2, observable=AVG)
    for prec in (F64, F32):
        a = bfi.bfi_eval(ctx, lat, prec, 5, sv, bfi.launch(32, 256, 0))
        b = bfi.bfi_eval(ctx, lat, prec, 5, sv, bfi.launch(32, 256, 1))
        assert np.array_equal(a, b)


def test_split_statistics(bfi, ctx):
    nx, nt = 10, 2
    sv = workloads.random_partition(20, 4.0, 6, per_sub=25_000, seed=11)
    for prec in (F64, F32):
        part, spl = bfi.bfi_eval(ctx, bfi.lattice(nx, nt, observable=AVG), prec, 3, sv, None,
                                 split=True)
        want = oracle.split_sums(oracle.lattice(nx, nt, observable=1), 3, sv.ids, sv.lo, sv.hi,
                                 sv.n, sv.offset)
        sig = spl[:, 0:1]
        got = np.concatenate([spl[:, 1:21] * np.exp(-sig), spl[:, 21:41] * np.exp(-2 * sig)], 1)
        tol = 1e-10 if prec == F64 else 1e-4
        tot = unshift(part, nx)
        scale = np.concatenate([np.repeat(tot[:, 1:2], 20, 1), np.repeat(tot[:, 2:3], 20, 1)], 1)
        assert np.all(np.abs(got - want) <= tol * scale)
        # the record of the split variant is the averaged record
        rec = oracle.sums(oracle.lattice(nx, nt, observable=1), 3, sv.ids, sv.lo, sv.hi, sv.n,
                          sv.offset)
        if prec == F64:
            assert_sums_close(tot, rec, nx, 1e-10)
        else:
            res_o = oracle.finalize(nx, 20, sv.lo, sv.hi, rec)
            assert_result_close(bfi.bfi_finalize(bfi.lattice(nx, nt, observable=AVG), sv, part),
                                res_o, 1e-4)


def test_10x2_full_size_sampled(bfi, ctx):
    """The benchmark workload (2^30 points, 1024 subvolumes) with the averaged
    product, in the benchmark's launch configuration (resident plan replayed as a
    graph); 4 subvolumes against the oracle, FP32 form against FP64."""
    w = workloads.WORKLOADS["burgers10x2"]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, w.budget // w.n_sub)
    lat = bfi.lattice(10, 2, observable=AVG)
    res = {}
    for prec in (F64, F32):
        plan = bfi.bfi_plan_create(ctx, lat, prec, sv, bfi.launch(use_graph=1))
        try:
            bfi.bfi_plan_run(plan, w.seed)
            got = bfi.bfi_plan_partials(plan, len(sv), 10)
        finally:
            bfi.bfi_plan_destroy(plan)
        res[prec] = bfi.bfi_finalize(lat, sv, got)
        if prec == F64:
            pick = np.array([0, 511, 700, 1023])
            sub = sv.subset(pick)
            want = oracle.sums(oracle.lattice(10, 2, observable=1), w.seed, sub.ids, sub.lo,
                               sub.hi, sub.n, sub.offset)
            assert_sums_close(unshift(got[pick], 10), want, 10, 1e-10)
    assert_result_close(res[F32], res[F64], 1e-4)
    # same points, anchored product: the same Z, consistent C(r)
    anch = bfi.bfi_integrate(ctx, bfi.lattice(10, 2), F64, w.seed, -w.box, w.box, w.split_log2,
                             w.budget)
    assert anch["Z"] == res[F64]["Z"]
    for r in range(10):
        both_err = np.hypot(anch["C_err"][r], res[F64]["C_err"][r])
        assert abs(anch["C"][r] - res[F64]["C"][r]) < 4 * both_err
        assert res[F64]["C"][r] == res[F64]["C"][(10 - r) % 10]


def test_variance_reduction_on_the_papers_range(bfi, ctx):
    """10x2 over the paper's integration range [-1, 1]^20 (section 4), 2^24
    points: on the same points the averaged product gives the anchored C(r)
    within the errors and a smaller error bar at every r."""
    lat_a = bfi.lattice(10, 2)
    lat_v = bfi.lattice(10, 2, observable=AVG)
    anch = bfi.bfi_integrate(ctx, lat_a, F64, 3, -1.0, 1.0, 6, 1 << 24)
    avg = bfi.bfi_integrate(ctx, lat_v, F64, 3, -1.0, 1.0, 6, 1 << 24)
    assert anch["Z"] == avg["Z"] and anch["ess"] > 1e4
    for r in range(10):
        assert abs(anch["C"][r] - avg["C"][r]) < 4 * anch["C_err"][r]
        assert avg["C_err"][r] < 0.8 * anch["C_err"][r], r


def test_16x4_sampled(bfi, ctx):
    w = workloads.WORKLOADS["burgers16x4"]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, 1 << 14)
    lat = bfi.lattice(16, 4, nu=0.5, observable=AVG)
    got = bfi.bfi_eval(ctx, lat, F64, w.seed, sv)
    pick = np.array([0, 2047, 4095])
    sub = sv.subset(pick)
    want = oracle.sums(oracle.lattice(16, 4, nu=0.5, observable=1), w.seed, sub.ids, sub.lo,
                       sub.hi, sub.n, sub.offset)
    assert_sums_close(unshift(got[pick], 16), want, 16, 1e-10)
    got32 = bfi.bfi_eval(ctx, lat, F32, w.seed, sv)
    assert_result_close(bfi.bfi_finalize(lat, sv, got32), bfi.bfi_finalize(lat, sv, got), 1e-4)


def test_adaptive_replays_on_oracle(bfi, ctx):
    nx, nt, B, nu = 3, 2, 2.0, 0.7
    cfg = bfi.adaptive_config(target_rel_err=1e-5, max_evals=1 << 21, n_min=1024,
                              n_max=1 << 16, split_log2=2, max_rounds=30, refine_fraction=0.5)
    out = bfi.bfi_integrate_adaptive(ctx, bfi.lattice(nx, nt, nu=nu, observable=AVG), "fp64", 3,
                                     -B, B, cfg)
    part = out["partition"]
    sums = oracle.sums(oracle.lattice(nx, nt, nu=nu, observable=1), 3, part.ids, part.lo, part.hi,
                       part.n, part.offset)
    ref = oracle.finalize(nx, nx * nt, part.lo, part.hi, sums)
    assert abs(out["Z"] - ref["Z"]) <= 1e-6 * ref["Z"]
    assert np.all(np.abs(out["C"] - ref["C"]) <= 1e-6 * abs(ref["C"][0]))


def test_served_mix_of_observables(bfi, ctx):
    """Requests that differ only in the observable run in separate groups of one
    step; each equals the oracle and is the same alone and in the mix."""
    srv = bfi.bfi_server_create(ctx, bfi.server_config(memory_budget=1 << 30))
    try:
        reqs = [bfi.request(bfi.lattice(4, 2, nu=0.5, observable=o), p, 7, 4.0, 4, 200_003)
                for o in ("anchor", AVG) for p in (F64, F32)]
        ts = [bfi.bfi_server_submit(srv, r) for r in reqs]
        mixed = [bfi.bfi_server_wait(srv, t, 60.0)[0] for t in ts]
    finally:
        bfi.bfi_server_destroy(srv)
    for i, obs in enumerate((0, 0, 1, 1)):
        ref = oracle.integrate_uniform(oracle.lattice(4, 2, nu=0.5, observable=obs), 7, -4.0, 4.0,
                                       4, 200_003)
        tol = 1e-6 if i % 2 == 0 else 1e-4
        assert abs(mixed[i]["Z"] - ref["Z"]) <= tol * ref["Z"]
        assert np.all(np.abs(mixed[i]["C"] - ref["C"]) <= tol * abs(ref["C"][0]))
    alone = bfi.bfi_server_create(ctx, bfi.server_config(memory_budget=1 << 30))
    try:
        one = bfi.bfi_server_wait(alone, bfi.bfi_server_submit(alone, reqs[2]), 60.0)[0]
    finally:
        bfi.bfi_server_destroy(alone)
    assert one["Z"] == mixed[2]["Z"] and np.array_equal(one["C"], mixed[2]["C"])


def test_integrand_correlation_averaged(bfi, ctx):
    nx, nt = 4, 2
    sv = workloads.uniform_partition(8, 2.0, 2, per_sub=5000)
    sums = oracle.sums(oracle.lattice(nx, nt, nu=0.8, observable=1), 4, sv.ids, sv.lo, sv.hi,
                       sv.n, sv.offset)
    V = np.prod(sv.hi - sv.lo, axis=1)
    f = bfi.integrand_burgers(bfi.lattice(nx, nt, nu=0.8, observable=AVG), F64, 1)
    n1, _, _ = bfi.bfi_integrand_eval(ctx, f, 4, sv)
    scale = V * np.sqrt(sums[:, 3 + nx + 1] * 5000) / 5000
    assert np.all(np.abs(n1 - V * sums[:, 3 + 1] / 5000) <= 1e-10 * scale)


def test_unknown_observable_rejected(bfi, ctx):
    sv = workloads.uniform_partition(8, 4.0, 1, per_sub=100)
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_eval(ctx, bfi.lattice(4, 2, observable=2), F64, 1, sv)
    assert e.value.name == "BFI_EINVAL"
