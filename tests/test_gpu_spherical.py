"""GPU parity of the sampler in spherical coordinates against the oracle on the
same seeded points, through the C ABI.

Bars: points within 1e-12 of the shell's outer radius (FP64; the two sides
take sines, cosines and the radius root by different routes) and 1e-4 of it in
the FP32 form; records within 1e-10 of each sum's Cauchy-Schwarz scale (the
oracle has no L1 sums for this sampler); Z (through log Z) within 1e-6 and
C(r) within 1e-6 of its Cauchy-Schwarz scale in FP64, 1e-4 in the FP32 form.
The two-stage integrator is replayed on the oracle (pilot records, the same
allocation, the continued streams); on 3x1 it meets Gauss-Legendre quadrature
within 4 sigma."""
import math

import numpy as np
import pytest

import oracle
from test_oracle_estimator import _gauss_legendre_box

pytestmark = pytest.mark.gpu


def _shells(d, B, k, n, offset=0):
    edges = np.linspace(0.0, B * math.sqrt(d), k + 1)
    ids = np.arange(1, k + 1, dtype=np.uint64)
    return ids, edges[:-1].copy(), edges[1:].copy(), n, offset


def _cs_scale_records(want, nx):
    """Cauchy-Schwarz scales of a plain sums record's fields (after n)."""
    n = want[:, 0:1]
    pw2 = want[:, 3 + nx:3 + 2 * nx]
    return np.concatenate([want[:, 1:3], np.sqrt(n * pw2), pw2,
                           np.sqrt(pw2) * np.sqrt(want[:, 2:3])], axis=1)


def _unshift(part, nx):
    f1 = np.exp(-part[:, 1])
    out = np.zeros((part.shape[0], 3 + 3 * nx))
    out[:, 0] = part[:, 0]
    out[:, 1] = part[:, 2] * f1
    out[:, 2] = part[:, 3] * f1**2
    out[:, 3:3 + nx] = part[:, 4:4 + nx] * f1[:, None]
    out[:, 3 + nx:] = part[:, 4 + nx:] * (f1**2)[:, None]
    return out


def _check(bfi, ctx, nx, nt, B, sh, seed, prec="fp64", params=None, launch=None):
    params = params or {}
    lat = bfi.lattice(nx, nt, **params)
    lat_o = oracle.lattice(nx, nt, **params)
    ids, lo, hi, n, off = sh
    print(f"sph: {nx}x{nt} {prec} {len(ids)} shells", flush=True)
    got = bfi.bfi_sph_eval(ctx, lat, prec, seed, B, bfi.Shells(ids, lo, hi, n, off), launch)
    want = oracle.sph_sums(lat_o, seed, B, ids, lo, hi, n, off)
    g = _unshift(got, nx)
    assert np.array_equal(g[:, 0], want[:, 0])
    d = nx * nt
    res_o = oracle.sph_finalize(nx, d, lo, hi, want)
    res_g = bfi.bfi_sph_finalize(lat, bfi.Shells(ids, lo, hi, n, off), got)
    tol = 1e-6 if prec == "fp64" else 1e-4
    if prec == "fp64":
        scale = _cs_scale_records(want, nx)
        err = np.abs(g[:, 1:] - want[:, 1:])
        assert np.all(err <= 1e-10 * scale + 1e-300), (err / (scale + 1e-300)).max()
    assert abs(res_g["log_Z"] - res_o["log_Z"]) <= tol
    # C(r) against the Cauchy-Schwarz bound of its L1 scale
    vol = np.array([oracle.sph_volume(d, a, b) for a, b in zip(lo, hi)])
    v = vol / want[:, 0]
    z = np.sum(v * want[:, 1])
    cs = np.sum(v[:, None] * np.sqrt(want[:, 0:1] * want[:, 3 + nx:3 + 2 * nx]), axis=0) / z
    assert np.all(np.abs(res_g["C"] - res_o["C"]) <= tol * (cs + np.abs(res_o["C"])))
    return got, res_g, res_o


@pytest.mark.parametrize("nx,nt", [(1, 1), (2, 1), (3, 1), (4, 2), (8, 2), (10, 2)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-4)])
def test_points_match_oracle(bfi, ctx, nx, nt, prec, tol):
    d = nx * nt
    lat = bfi.lattice(nx, nt)
    idx = np.array([0, 1, 2, 17, 1023, 2**20 + 5, 2**33 + 7], dtype=np.uint64)
    for sid, seed, a, b in ((1, 1, 0.0, 1.5), (9, 3, 2.0, 2.5), (2**40 + 3, 7, 0.5, 9.0)):
        got = bfi.bfi_debug_sph_points(ctx, lat, prec, seed, sid, a, b, idx)
        want = np.stack([oracle.sph_point(d, seed, sid, a, b, int(i)) for i in idx])
        assert np.all(np.abs(got - want) <= tol * b), (sid, np.abs(got - want).max() / b)


@pytest.mark.parametrize("nx,nt,B", [(3, 1, 2.0), (4, 2, 1.0), (10, 2, 1.0), (10, 2, 4.0),
                                     (5, 3, 1.5)])
def test_records_match_oracle(bfi, ctx, nx, nt, B):
    d = nx * nt
    sh = _shells(d, B, 8, 1, 0)
    n = np.array([2, 3, 257, 65536 + 3, 4000, 70001, 999, 1 << 14], dtype=np.uint64)
    off = np.array([0, 5, 2**20, 3, 0, 2**33, 1, 7], dtype=np.uint64)
    _check(bfi, ctx, nx, nt, B, (sh[0], sh[1], sh[2], n, off), 11, params=dict(nu=0.8))
    _check(bfi, ctx, nx, nt, B, (sh[0], sh[1], sh[2], n, off), 11, "fp32", params=dict(nu=0.8))


def test_averaged_observable_and_launch_shapes(bfi, ctx):
    sh = _shells(20, 1.0, 6, 20000)
    _check(bfi, ctx, 10, 2, 1.0, sh, 3, params=dict(observable=1))
    lat = bfi.lattice(10, 2)
    shells = bfi.Shells(*sh)
    grid = bfi.bfi_sph_eval(ctx, lat, "fp64", 3, 1.0, shells,
                            bfi.launch(samples_per_thread=16, block=64, persistent=0))
    pers = bfi.bfi_sph_eval(ctx, lat, "fp64", 3, 1.0, shells,
                            bfi.launch(samples_per_thread=16, block=64, persistent=1))
    assert np.array_equal(grid.view(np.uint64), pers.view(np.uint64))
    _check(bfi, ctx, 10, 2, 1.0, sh, 3, launch=bfi.launch(samples_per_thread=7, block=128,
                                                          persistent=1))


def test_two_stage_integrator_replays_on_oracle(bfi, ctx):
    """Pilot records, then the rest of the budget in proportion to shell volume
    times the pilot's spread of the weight, each shell continuing its stream."""
    nx, nt, B = 3, 1, 2.0
    d = nx * nt
    k, budget, frac = 8, 1 << 17, 0.25
    lat = bfi.lattice(nx, nt)
    res = bfi.bfi_integrate_sph(ctx, lat, "fp64", 5, B, k, budget, frac)
    lat_o = oracle.lattice(nx, nt)
    ids, lo, hi, _, _ = _shells(d, B, k, 1)
    pilot = int(frac * budget) // k
    p = oracle.sph_sums(lat_o, 5, B, ids, lo, hi, pilot, 0)
    vol = np.array([oracle.sph_volume(d, a, b) for a, b in zip(lo, hi)])
    sd = np.sqrt(np.maximum(p[:, 2] / pilot - (p[:, 1] / pilot) ** 2, 0.0))
    share = vol * sd
    rest = budget - pilot * k
    main = np.floor(share / share.sum() * rest).astype(np.uint64)
    sums = p.copy()
    take = main >= 2
    if take.any():
        m = oracle.sph_sums(lat_o, 5, B, ids[take], lo[take], hi[take], main[take], pilot)
        sums[take] += m
    ref = oracle.sph_finalize(nx, d, lo, hi, sums)
    assert res["n_evals"] == sums[:, 0].sum()
    assert abs(res["log_Z"] - ref["log_Z"]) < 1e-9
    np.testing.assert_allclose(res["C"], ref["C"], rtol=1e-8, atol=1e-10)
    # and the estimate meets quadrature
    Zq, Cq = _gauss_legendre_box(lat_o, B, 8)
    assert abs(res["Z"] - Zq) < 4 * res["Z_err"]
    for r in range(nx):
        assert abs(res["C"][r] - Cq[r]) < 4 * res["C_err"][r]


def test_fp32_form_integrator_agrees(bfi, ctx):
    lat = bfi.lattice(4, 2)
    r64 = bfi.bfi_integrate_sph(ctx, lat, "fp64", 1, 1.0, 16, 1 << 20)
    r32 = bfi.bfi_integrate_sph(ctx, lat, "fp32", 1, 1.0, 16, 1 << 20)
    assert abs(r32["log_Z"] - r64["log_Z"]) < 1e-4
    assert np.all(np.abs(r32["C"] - r64["C"]) < 1e-4 * np.abs(r64["C"][0]) + 3 * r64["C_err"])


def test_refusals(bfi, ctx):
    sh = bfi.Shells([1], [0.0], [1.0], [100])
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_sph_eval(ctx, bfi.lattice(4, 2), "fp64s", 1, 1.0, sh)
    assert e.value.status == -4
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_sph_eval(ctx, bfi.lattice(4, 2, antithetic=True), "fp64", 1, 1.0, sh)
    assert e.value.status == -4
    with pytest.raises(bfi.BfiError) as e:
        bfi.bfi_sph_eval(ctx, bfi.lattice(16, 4), "fp64", 1, 1.0, sh)
    assert e.value.status == -4
    for bad in (bfi.Shells([1], [1.0], [1.0], [100]), bfi.Shells([1], [0.0], [1.0], [1]),
                bfi.Shells([1], [-0.5], [1.0], [100])):
        with pytest.raises(bfi.BfiError) as e:
            bfi.bfi_sph_eval(ctx, bfi.lattice(4, 2), "fp64", 1, 1.0, bad)
        assert e.value.status == -1
    with pytest.raises(bfi.BfiError):
        bfi.bfi_sph_eval(ctx, bfi.lattice(4, 2), "fp64", 1, 0.0, sh)
    with pytest.raises(bfi.BfiError):
        bfi.bfi_integrate_sph(ctx, bfi.lattice(4, 2), "fp64", 1, 1.0, 64, 100)
