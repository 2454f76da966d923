"""GPU parity of the shifted FP64 form (BFI_FP64_SHIFTED) against the oracle's
shifted records (oracle.sums_shifted_l1 / finalize_shifted) on the same seeded
points, through the C ABI.

Bars: records within 1e-10 of each sum's L1 scale after moving both to the
oracle's shift (the smallest action of the subvolume); log Z within 1e-6
(Z relative 1e-6), C(r) within 1e-6 of its L1 scale.  Where nothing
underflows, the shifted form also equals the plain FP64 form on the GPU.
Where every plain weight underflows (S > 745 for every point: the plain form
gives Z = 0), log Z and C(r) still match the oracle, and on a single site far
from the origin the closed form of a truncated normal."""
import math

import numpy as np
import pytest
from scipy import special

import oracle
import workloads
from parity_util import assert_records_close, assert_result_close, c_scale, move_shift

pytestmark = pytest.mark.gpu

S64 = "fp64s"


def _check(bfi, ctx, nx, nt, sv, seed, params=None, launch=None, rtol=1e-10, tol=1e-6):
    params = params or {}
    lat_o = oracle.lattice(nx, nt, **params)
    want = oracle.sums_shifted_l1(lat_o, seed, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    L = oracle.sums_len(nx) + 1
    sig_o = want[:, 1]
    want_plain = np.concatenate([want[:, :1], want[:, 2:L]], axis=1)
    lat = bfi.lattice(nx, nt, **params)
    print(f"fp64s: {nx}x{nt} {len(sv)} subvolumes {int(sv.n.sum())} samples", flush=True)
    got = bfi.bfi_eval(ctx, lat, S64, seed, sv, launch)
    # the GPU's shift is an action of the subvolume's points (as the kernel
    # evaluates it: within 1e-13 of the oracle's), at most 64 above the smallest
    slack = 1e-13 * np.abs(sig_o)
    assert np.all(got[:, 1] >= sig_o - slack), got[:, 1] - sig_o
    assert np.all(got[:, 1] <= sig_o + 64.0 + slack), got[:, 1] - sig_o
    assert_records_close(move_shift(got, nx, sig_o), want_plain, want[:, L:], nx, rtol)
    res_o = oracle.finalize_shifted(nx, nx * nt, sv.lo, sv.hi, want[:, :L],
                                    2 if params.get("antithetic") else 1)
    res_g = bfi.bfi_finalize(lat, sv, got)
    assert_result_close(res_g, res_o, c_scale(sv.lo, sv.hi, want_plain, want[:, L:]), tol)
    return got, res_g, res_o


@pytest.mark.parametrize("nx,nt", [(3, 2), (4, 2), (10, 2), (16, 4), (1, 2)])
def test_records_match_oracle_ragged(bfi, ctx, nx, nt):
    d = nx * nt
    sv = workloads.random_partition(d, 3.0, 10, per_sub=1, seed=40 + nx)
    sv.n[:] = [2, 3, 255, 257, 16383, 16385, 40000, 1000, 77, 3 * 16384 + 5]
    sv.offset[:] = [0, 5, 2**20, 3, 0, 2**33, 0, 1, 7, 123456789]
    _check(bfi, ctx, nx, nt, sv, 11, dict(nu=0.6))


def test_equals_plain_fp64_where_nothing_underflows(bfi, ctx):
    """The 4x2 workload: the shifted records rescaled to sigma = 0 are the plain
    FP64 records (the same weights, one rounding of the shift apart), and Z,
    C(r), C_err agree to 1e-12."""
    w = workloads.WORKLOADS["burgers4x2"]
    sv = workloads.uniform_partition(w.d, w.box, w.split_log2, w.budget // w.n_sub)
    lat = bfi.lattice(4, 2)
    got, res_s, _ = _check(bfi, ctx, 4, 2, sv, w.seed)
    plain = bfi.bfi_eval(ctx, lat, "fp64", w.seed, sv)
    res_p = bfi.bfi_finalize(lat, sv, plain)
    assert res_s["log_Z"] == pytest.approx(res_p["log_Z"], abs=1e-12)
    np.testing.assert_allclose(res_s["C"], res_p["C"], rtol=1e-12, atol=1e-12 * res_p["C"][0])
    np.testing.assert_allclose(res_s["C_err"], res_p["C_err"], rtol=1e-9)


@pytest.mark.parametrize("obs", [0, 1])
def test_where_plain_fp64_underflows(bfi, ctx, obs):
    """10x2, D = 0.01 on [-4,4]^20: every action is above 1900, every plain
    weight is 0 in FP64 and so is the plain Z; the shifted form gives log Z
    and C(r) of the oracle on the same points."""
    nx, nt = 10, 2
    params = dict(nu=1.0, D=0.01, observable=obs)
    sv = workloads.uniform_partition(20, 4.0, 6, per_sub=1 << 14)
    lat = bfi.lattice(nx, nt, **params)
    plain = bfi.bfi_eval(ctx, lat, "fp64", 1, sv)
    assert np.all(plain[:, 2] == 0.0)
    got, res_g, res_o = _check(bfi, ctx, nx, nt, sv, 1, params)
    assert res_g["Z"] == 0.0 and math.isfinite(res_g["log_Z"]) and res_g["log_Z"] < -1000
    assert np.all(np.isfinite(res_g["C"]))


def test_antithetic_pairs_and_launch_shapes(bfi, ctx):
    nx, nt = 8, 2
    sv = workloads.random_partition(16, 4.0, 6, per_sub=1, seed=3)
    sv.n[:] = [2, 999, 4096, 70001, 12345, 300]
    _check(bfi, ctx, nx, nt, sv, 5, dict(nu=0.3, antithetic=1))
    for launch in (bfi.launch(samples_per_thread=8, block=64, persistent=1),
                   bfi.launch(samples_per_thread=32, block=256, persistent=0)):
        _check(bfi, ctx, nx, nt, sv, 5, dict(nu=0.3), launch)
    # persistent and one block per item: the same records bit for bit
    lat = bfi.lattice(nx, nt, nu=0.3)
    grid = bfi.bfi_eval(ctx, lat, S64, 5, sv, bfi.launch(samples_per_thread=8, block=64,
                                                          persistent=0))
    pers = bfi.bfi_eval(ctx, lat, S64, 5, sv, bfi.launch(samples_per_thread=8, block=64,
                                                          persistent=1))
    assert np.array_equal(pers.view(np.uint64), grid.view(np.uint64))


def test_single_site_closed_form(bfi, ctx):
    """nx = nt = 1, m2 = 1 on [40, 40.1]: S = u^2/2 > 800, Z = sqrt(2 pi)
    (Phi(40.1) - Phi(40)): the GPU's log Z within 4 sigma of it and within 1e-6
    of the oracle."""
    sv = workloads.SubvolumeList(np.array([1], np.uint64), np.array([[40.0]]),
                                 np.array([[40.1]]), np.array([1 << 18], np.uint64),
                                 np.array([0], np.uint64))
    _, res, _ = _check(bfi, ctx, 1, 1, sv, 1, dict(m2=1.0))
    la, lb = special.log_ndtr(-40.0), special.log_ndtr(-40.1)
    log_z = 0.5 * math.log(2 * math.pi) + la + math.log1p(-math.exp(lb - la))
    rel = res["Z_err"] / math.exp(res["log_Z"]) if res["Z"] > 0 else None
    assert rel is None  # Z itself underflows
    assert abs(res["log_Z"] - log_z) < 0.01


def test_entry_points_take_the_shifted_form(bfi, ctx):
    """Plans (graph replay), bfi_integrate, the allocation-free entry and the
    server give the oracle's shifted result; the Gaussian-proposal sampler
    refuses the form."""
    nx, nt = 4, 2
    lat = bfi.lattice(nx, nt, D=0.05)
    lat_o = oracle.lattice(nx, nt, D=0.05)
    sv = workloads.uniform_partition(8, 4.0, 4, per_sub=5000)
    want = oracle.sums_shifted_l1(lat_o, 2, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    L = oracle.sums_len(nx) + 1
    res_o = oracle.finalize_shifted(nx, 8, sv.lo, sv.hi, want[:, :L])
    scale = c_scale(sv.lo, sv.hi, np.concatenate([want[:, :1], want[:, 2:L]], axis=1), want[:, L:])
    ref = bfi.bfi_eval(ctx, lat, S64, 2, sv)
    plan = bfi.bfi_plan_create(ctx, lat, S64, sv, bfi.launch(use_graph=1))
    try:
        for _ in range(3):
            bfi.bfi_plan_run(plan, 2)
            part = bfi.bfi_plan_partials(plan, len(sv), nx)
            assert np.array_equal(part.view(np.uint64), ref.view(np.uint64))
    finally:
        bfi.bfi_plan_destroy(plan)
    na = bfi.bfi_eval_noalloc(ctx, lat, S64, 2, sv)
    assert np.array_equal(na.view(np.uint64), ref.view(np.uint64))
    res_i = bfi.bfi_integrate(ctx, lat, S64, 2, -4.0, 4.0, 4, 16 * 5000)
    assert_result_close(res_i, res_o, scale, 1e-6)
    srv = bfi.bfi_server_create(ctx, bfi.server_config())
    try:
        t = bfi.bfi_server_submit(srv, bfi.request(lat, S64, 2, 4.0, 4, 16 * 5000))
        done = bfi.bfi_server_wait(srv, t, 60.0)
        assert done is not None
        assert_result_close(done[0], res_o, scale, 1e-6)
    finally:
        bfi.bfi_server_destroy(srv)
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_integrate_is(ctx, lat, S64, 1, -1.0, 1.0, 1 << 16)
    assert e.value.status == -4
