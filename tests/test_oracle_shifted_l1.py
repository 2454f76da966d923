"""Pins of the oracle's L1-scale sums and shifted weights (CPU only).

* oracle_sums_l1: the first fields are oracle_sums' own record bit for bit; the
  extra fields are sum |p_r w| -- brute force over the pinned point, action and
  observable, equal to the signed sums where every product is positive, and
  never below their absolute value; for antithetic pairs, the absolute value of
  the pair mean.
* oracle_sums_shifted / oracle_finalize_shifted: the shift is the smallest
  action of the subvolume's points (brute force); rescaled by exp(-sigma) the
  records are the plain ones wherever nothing underflows, and so is the
  finalize; where every plain weight underflows (Z = 0 in FP64), log Z and C(0)
  match closed forms: a single site with a mass term far from the origin
  (S = m2 u^2 / 2, a truncated normal) and two sites whose difference is
  confined away from 0 (S = 4 nu^2 tau (u1 - u0)^2 / (D a^4), 2-D quadrature).
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle
import workloads


def _records(lat, sv, seed, fn):
    return fn(lat, seed, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)


@pytest.mark.parametrize("nx,nt,obs", [(4, 2, 0), (3, 2, 1), (5, 1, 0)])
def test_l1_extends_the_sums_record(nx, nt, obs):
    lat = oracle.lattice(nx, nt, nu=0.7, observable=obs)
    sv = workloads.random_partition(nx * nt, 2.0, 6, per_sub=700, seed=nx)
    plain = _records(lat, sv, 5, oracle.sums)
    l1 = _records(lat, sv, 5, oracle.sums_l1)
    L = oracle.sums_len(nx)
    assert np.array_equal(l1[:, :L].view(np.uint64), plain.view(np.uint64))
    assert np.all(l1[:, L:] >= np.abs(plain[:, 3:3 + nx]))
    assert np.all(l1[:, L:] <= np.sqrt(plain[:, 0:1] * plain[:, 3 + nx:3 + 2 * nx]) * (1 + 1e-12))


def test_l1_brute_force():
    nx, nt = 3, 2
    d = nx * nt
    lat = oracle.lattice(nx, nt, nu=0.4)
    sv = workloads.random_partition(d, 1.5, 3, per_sub=257, seed=2)
    sv.offset[:] = [0, 11, 2**33]
    got = _records(lat, sv, 9, oracle.sums_l1)
    for s in range(len(sv)):
        idx = int(sv.offset[s]) + np.arange(int(sv.n[s]))
        u = oracle.points(d, 9, int(sv.ids[s]), sv.lo[s], sv.hi[s], idx)
        w = np.exp(-oracle.action_batch(lat, u))
        p = np.stack([oracle.observable(lat, x) for x in u])
        want = np.abs(p * w[:, None]).sum(axis=0)
        np.testing.assert_allclose(got[s, 3 + 3 * nx:], want, rtol=1e-12)


def test_l1_equals_signed_sums_in_the_positive_orthant():
    """Every coordinate positive: every anchored product is positive, so the
    L1 field and the signed sum are the same Neumaier sum of the same terms."""
    lat = oracle.lattice(4, 2, nu=1.0)
    sv = workloads.uniform_partition(8, 1.0, 3, per_sub=2000)
    sv.lo[:] = sv.lo + 1.5  # [0.5, 2.5] before the split, all coordinates > 0
    sv.hi[:] = sv.hi + 1.5
    got = _records(lat, sv, 1, oracle.sums_l1)
    assert np.array_equal(got[:, 3 + 12:], got[:, 3:3 + 4])


def test_l1_of_antithetic_pairs_brute_force():
    nx, nt = 2, 2
    d = nx * nt
    lat = oracle.lattice(nx, nt, nu=0.9, antithetic=1)
    lo, hi = np.array([[-1.0, 0.0, -2.0, 0.5]]), np.array([[1.0, 2.0, 0.0, 1.5]])
    got = oracle.sums_l1(lat, 4, [5], lo, hi, [300], [7])
    single = oracle.lattice(nx, nt, nu=0.9)
    idx = 7 + np.arange(300)
    wa, wb, pa, pb = [], [], [], []
    for i in idx:
        x = oracle.words(d, 4, 5, int(i)).astype(np.float64)
        scale = (hi[0] - lo[0]) * 2.0**-32
        base = lo[0] + 0.5 * scale
        ua = x * scale + base
        ub = (4294967295.0 - x) * scale + base
        wa.append(math.exp(-oracle.action(single, ua)))
        wb.append(math.exp(-oracle.action(single, ub)))
        pa.append(oracle.observable(single, ua))
        pb.append(oracle.observable(single, ub))
    wa, wb, pa, pb = map(np.asarray, (wa, wb, pa, pb))
    want = np.abs(0.5 * (pa * wa[:, None] + pb * wb[:, None])).sum(axis=0)
    np.testing.assert_allclose(got[0, 3 + 3 * nx:], want, rtol=1e-10)


@pytest.mark.parametrize("anti", [0, 1])
def test_shift_is_the_smallest_action_and_rescales_to_plain(anti):
    nx, nt = 4, 2
    d = nx * nt
    lat = oracle.lattice(nx, nt, nu=0.8, antithetic=anti)
    sv = workloads.random_partition(d, 3.0, 5, per_sub=600, seed=3)
    sh = _records(lat, sv, 2, oracle.sums_shifted)
    plain = _records(lat, sv, 2, oracle.sums)
    single = oracle.lattice(nx, nt, nu=0.8)
    for s in range(len(sv)):
        idx = np.arange(int(sv.n[s]))
        u = oracle.points(d, 2, int(sv.ids[s]), sv.lo[s], sv.hi[s], idx)
        S = oracle.action_batch(single, u)
        if anti:
            ub = sv.lo[s] + sv.hi[s] - u  # the reflection (exact on these dyadic boxes)
            S = np.concatenate([S, oracle.action_batch(single, ub)])
        assert sh[s, 1] == S.min()
    f1 = np.exp(-sh[:, 1])[:, None]
    nx3 = 3 * nx
    assert np.array_equal(sh[:, 0], plain[:, 0])
    np.testing.assert_allclose(sh[:, 2:3] * f1, plain[:, 1:2], rtol=1e-13)
    np.testing.assert_allclose(sh[:, 3:4] * f1**2, plain[:, 2:3], rtol=1e-13)
    np.testing.assert_allclose(sh[:, 4:4 + nx] * f1, plain[:, 3:3 + nx], rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(sh[:, 4 + nx:4 + nx3] * f1**2, plain[:, 3 + nx:3 + nx3],
                               rtol=1e-12, atol=1e-300)
    ref = oracle.finalize(nx, d, sv.lo, sv.hi, plain, 2 if anti else 1)
    got = oracle.finalize_shifted(nx, d, sv.lo, sv.hi, sh, 2 if anti else 1)
    assert got["log_Z"] == pytest.approx(ref["log_Z"], abs=1e-13)
    assert got["Z"] == pytest.approx(ref["Z"], rel=1e-12)
    assert got["Z_err"] == pytest.approx(ref["Z_err"], rel=1e-10)
    assert got["ess"] == pytest.approx(ref["ess"], rel=1e-12)
    assert got["n_evals"] == ref["n_evals"]
    np.testing.assert_allclose(got["C"], ref["C"], rtol=1e-12)
    np.testing.assert_allclose(got["C_err"], ref["C_err"], rtol=1e-10)


def test_finalize_shifted_moves_records_to_the_smallest_shift():
    """Adding c to a record's shift and multiplying its first-order sums by
    exp(c) (second-order by exp(2c)) describes the same sums: the result does
    not change."""
    lat = oracle.lattice(3, 2, nu=0.5)
    sv = workloads.uniform_partition(6, 2.0, 2, per_sub=500)
    sh = _records(lat, sv, 8, oracle.sums_shifted)
    ref = oracle.finalize_shifted(3, 6, sv.lo, sv.hi, sh)
    moved = sh.copy()
    for s, c in enumerate([3.0, -7.5, 0.0, 40.0]):
        moved[s, 1] += c
        moved[s, 2] *= math.exp(c)
        moved[s, 3] *= math.exp(2 * c)
        moved[s, 4:7] *= math.exp(c)
        moved[s, 7:13] *= math.exp(2 * c)
    got = oracle.finalize_shifted(3, 6, sv.lo, sv.hi, moved)
    assert got["log_Z"] == pytest.approx(ref["log_Z"], abs=1e-12)
    np.testing.assert_allclose(got["C"], ref["C"], rtol=1e-11)
    np.testing.assert_allclose(got["C_err"], ref["C_err"], rtol=1e-10)


def _log_norm_interval(a, b):
    """log(Phi(b) - Phi(a)) for 0 < a < b, from the upper tails."""
    la, lb = special.log_ndtr(-a), special.log_ndtr(-b)
    return la + math.log1p(-math.exp(lb - la))


def _rel_err_of_mean(sum_w, sum_w2, n):
    return math.sqrt(max(sum_w2 / sum_w**2 - 1.0 / n, 0.0) * n / (n - 1))


def test_single_site_far_from_origin_closed_form():
    """nx = nt = 1: the time difference, the advection and the viscosity terms
    vanish (periodic wrap onto the same site), S = m2 u^2 / 2.  On [40, 40.1]
    every weight is below exp(-800), so the plain FP64 sums are 0; the shifted
    ones give log Z = log(sqrt(2 pi) (Phi(40.1) - Phi(40))) and C(0) = <u^2> of
    the truncated normal, 1 + (a phi(a) - b phi(b)) / (Phi(b) - Phi(a)).  The
    weight falls by about e^4 across the box, so the error bars hold."""
    a, b = 40.0, 40.1
    lat = oracle.lattice(1, 1, m2=1.0)
    ids = np.array([1], dtype=np.uint64)
    lo, hi = np.array([[a]]), np.array([[b]])
    n = 1 << 18
    assert oracle.sums(lat, 1, ids, lo, hi, [n])[0, 1] == 0.0  # every plain weight underflows
    sh = oracle.sums_shifted(lat, 1, ids, lo, hi, [n])
    assert sh[0, 1] > 800.0
    res = oracle.finalize_shifted(1, 1, lo, hi, sh)
    assert res["Z"] == 0.0 and math.isfinite(res["log_Z"])
    log_mass = _log_norm_interval(a, b)
    log_z = 0.5 * math.log(2 * math.pi) + log_mass
    rel = _rel_err_of_mean(sh[0, 2], sh[0, 3], n)
    assert rel < 0.01
    assert abs(res["log_Z"] - log_z) <= 4 * rel
    log_phi = lambda x: -0.5 * x * x - 0.5 * math.log(2 * math.pi)  # noqa: E731
    c0 = 1.0 + a * math.exp(log_phi(a) - log_mass) - b * math.exp(log_phi(b) - log_mass)
    assert abs(res["C"][0] - c0) <= 4 * res["C_err"][0]
    assert res["C_err"][0] < 1e-3 * c0


def test_two_sites_far_apart_quadrature():
    """nx = 2, nt = 1: S = 4 nu^2 tau (u1 - u0)^2 / (D a^4) (the advection term
    cancels on two sites); with D = 4, S = (u1 - u0)^2.  u0 in [0, 0.05] and
    u1 in [28, 28.05] put S in [781, 787]: plain FP64 gives Z = 0.  Z, <u0 u0>
    and <u0 u1> from 2-D quadrature of exp(784 - S) over the box, which varies
    by about e^3."""
    lat = oracle.lattice(2, 1, D=4.0)
    ids = np.array([1], dtype=np.uint64)
    lo, hi = np.array([[0.0, 28.0]]), np.array([[0.05, 28.05]])
    n = 1 << 18
    assert oracle.sums(lat, 3, ids, lo, hi, [n])[0, 1] == 0.0
    sh = oracle.sums_shifted(lat, 3, ids, lo, hi, [n])
    res = oracle.finalize_shifted(2, 2, lo, hi, sh)
    assert res["Z"] == 0.0

    def moment(h):
        val, _ = integrate.dblquad(lambda u1, u0: h(u0, u1) * math.exp(784.0 - (u1 - u0) ** 2),
                                   0.0, 0.05, 28.0, 28.05, epsabs=0, epsrel=1e-12)
        return val

    z0 = moment(lambda x, y: 1.0)
    log_z = -784.0 + math.log(z0)
    rel = _rel_err_of_mean(sh[0, 2], sh[0, 3], n)
    assert rel < 0.01
    assert abs(res["log_Z"] - log_z) <= 4 * rel
    for r, h in ((0, lambda x, y: x * x), (1, lambda x, y: x * y)):
        c = moment(h) / z0
        assert abs(res["C"][r] - c) <= 4 * res["C_err"][r], (r, res["C"][r], c, res["C_err"][r])
        assert res["C_err"][r] < 0.02 * abs(c)


def test_shifted_l1_is_both_records():
    """The shifted record with L1 fields: its first fields are oracle_sums_shifted's
    record bit for bit, and its L1 fields times exp(-sigma) are oracle_sums_l1's."""
    nx, nt = 3, 2
    lat = oracle.lattice(nx, nt, nu=0.6)
    sv = workloads.random_partition(nx * nt, 2.5, 4, per_sub=900, seed=7)
    both = _records(lat, sv, 6, oracle.sums_shifted_l1)
    sh = _records(lat, sv, 6, oracle.sums_shifted)
    l1 = _records(lat, sv, 6, oracle.sums_l1)
    L = oracle.sums_len(nx) + 1
    assert np.array_equal(both[:, :L].view(np.uint64), sh.view(np.uint64))
    np.testing.assert_allclose(both[:, L:] * np.exp(-both[:, 1:2]), l1[:, L - 1:], rtol=1e-12)
