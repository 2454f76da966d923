"""Pins for the oracle's antithetic pairs (the plain estimate of section 3 with
antithetic variates): sample index i gives the point u of its Philox words x and
the point u' of the complemented words 0xFFFFFFFF - x; records run over pairs
with w -> (w(u) + w(u'))/2 and p_r w -> (p_r(u) w(u) + p_r(u') w(u'))/2.

  * the partner is the reflection of u through the subvolume's centre, exactly,
    on dyadic boxes (numpy arithmetic on the words);
  * g = 0 on a box centred at 0: u' = -u and S(-u) = S(u) bit for bit, so the
    pair record is the plain record of the same indices, field for field;
  * g = 1 on a centred box: S(-u; g) = S(u; -g) bit for bit, so the first-order
    sums are the means of the plain sums at g and at -g;
  * brute force over pairs on a subvolume that is not centred (numpy products
    and sums over the oracle's pinned action);
  * statistics: the pair estimate agrees with the plain one, and on the
    subvolumes of a partition (not centred) its error bar at equal evaluations
    is the plain one's (the two weights of a pair are nearly uncorrelated there);
  * pairs have no split statistics."""
import math

import numpy as np
import pytest

import oracle
import workloads


def dyadic_sub(d, seed):
    sv = workloads.random_partition(d, 2.0, 6, per_sub=1, seed=seed)
    return sv.subset(np.array([3]))


@pytest.mark.parametrize("d", [1, 5, 8, 20])
def test_partner_is_the_reflection(oracle_lib, d):
    sub = dyadic_sub(d, d)
    lo, hi = sub.lo[0], sub.hi[0]
    scale = (hi - lo) * 2.0**-32
    base = lo + 0.5 * scale
    for i in [0, 1, 7, 2**33 + 5]:
        x = oracle.words(d, 3, int(sub.ids[0]), i).astype(np.float64)
        u = oracle.point(d, 3, int(sub.ids[0]), lo, hi, i)
        # x scale is exact on a dyadic box, so base + x scale is the fma
        np.testing.assert_array_equal(u, base + x * scale)
        ub = base + (4294967295.0 - x) * scale
        np.testing.assert_array_equal(ub, lo + hi - u)
        assert np.all((lo < ub) & (ub < hi))


@pytest.mark.parametrize("obs", [0, 1])
@pytest.mark.parametrize("nx,nt", [(3, 2), (4, 2), (10, 2)])
def test_gaussian_centred_box_pairs_are_plain_records(oracle_lib, nx, nt, obs):
    d = nx * nt
    B = 1.5
    ids = np.array([1, 2, 3], np.uint64)
    lo, hi = np.full((3, d), -B), np.full((3, d), B)
    plain = oracle.sums(oracle.lattice(nx, nt, nu=0.7, g=0.0, observable=obs), 5, ids, lo, hi,
                        700, [0, 9, 2**40])
    pair = oracle.sums(oracle.lattice(nx, nt, nu=0.7, g=0.0, observable=obs, antithetic=1), 5,
                       ids, lo, hi, 700, [0, 9, 2**40])
    np.testing.assert_array_equal(pair, plain)


@pytest.mark.parametrize("nx,nt", [(3, 2), (5, 3), (10, 2)])
def test_centred_box_first_order_is_mean_over_g_signs(oracle_lib, nx, nt):
    d = nx * nt
    ids = np.array([1, 6], np.uint64)
    lo, hi = np.full((2, d), -2.0), np.full((2, d), 2.0)
    args = (7, ids, lo, hi, 3000, 0)
    plus = oracle.sums(oracle.lattice(nx, nt, nu=0.6, g=1.0), *args)
    minus = oracle.sums(oracle.lattice(nx, nt, nu=0.6, g=-1.0), *args)
    pair = oracle.sums(oracle.lattice(nx, nt, nu=0.6, g=1.0, antithetic=1), *args)
    first = [1] + list(range(3, 3 + nx))
    want = 0.5 * (plus[:, first] + minus[:, first])
    np.testing.assert_allclose(pair[:, first], want, rtol=1e-13, atol=0)
    assert np.array_equal(pair[:, 0], plus[:, 0])
    # second order: the pair mean squared lies between 0 and the mean of squares
    assert np.all(pair[:, 2] <= 0.5 * (plus[:, 2] + minus[:, 2]) * (1 + 1e-13))


@pytest.mark.parametrize("obs", [0, 1])
@pytest.mark.parametrize("nx,nt", [(3, 1), (3, 2), (4, 2)])
def test_brute_force_over_pairs(oracle_lib, nx, nt, obs):
    d = nx * nt
    sub = dyadic_sub(d, 10 * nx + nt)
    lo, hi, sid = sub.lo[0], sub.hi[0], int(sub.ids[0])
    lat_plain = oracle.lattice(nx, nt, nu=0.8, observable=obs)
    idx = np.arange(11, 11 + 40)
    u = oracle.points(d, 2, sid, lo, hi, idx)
    ub = lo + hi - u                       # exact on a dyadic box (test above)
    w = np.exp(-oracle.action_batch(lat_plain, u))
    wb = np.exp(-oracle.action_batch(lat_plain, ub))

    def prods(v):
        f = v.reshape(-1, nt, nx)
        if obs == 0:
            return f[:, 0, :1] * f[:, 0, :]
        return np.stack([(f * np.roll(f, -r, axis=2)).mean(axis=(1, 2)) for r in range(nx)], 1)

    W = 0.5 * (w + wb)
    P = 0.5 * (prods(u) * w[:, None] + prods(ub) * wb[:, None])
    want = np.concatenate([[len(idx), W.sum(), (W * W).sum()], P.sum(0), (P * P).sum(0),
                           (P * W[:, None]).sum(0)])
    got = oracle.sums(oracle.lattice(nx, nt, nu=0.8, observable=obs, antithetic=1), 2,
                      [sid], lo[None], hi[None], len(idx), 11)[0]
    scale = np.concatenate([[1, W.sum(), (W * W).sum()], np.abs(P).sum(0), (P * P).sum(0),
                            np.abs(P * W[:, None]).sum(0)])
    assert np.all(np.abs(got - want) <= 1e-13 * scale)


def test_pairs_agree_with_plain_and_match_its_error_on_subvolumes(oracle_lib):
    """4x2, nu = 1, [-2,2]^8 in 64 subvolumes: 2^13 pairs per subvolume against
    2^14 plain samples (same evaluations)."""
    nx, nt = 4, 2
    sv = workloads.uniform_partition(8, 2.0, 6, per_sub=1 << 14)
    plain = oracle.finalize(nx, 8, sv.lo, sv.hi,
                            oracle.sums(oracle.lattice(nx, nt), 1, sv.ids, sv.lo, sv.hi, sv.n, 0))
    pl = oracle.lattice(nx, nt, antithetic=1)
    pair = oracle.finalize(nx, 8, sv.lo, sv.hi,
                           oracle.sums(pl, 2, sv.ids, sv.lo, sv.hi, sv.n // 2, 0), 2)
    assert pair["n_evals"] == plain["n_evals"]
    assert abs(pair["Z"] - plain["Z"]) < 4 * math.hypot(pair["Z_err"], plain["Z_err"])
    for r in range(nx):
        assert abs(pair["C"][r] - plain["C"][r]) < 4 * math.hypot(pair["C_err"][r],
                                                                   plain["C_err"][r])
    assert 0.8 < pair["Z_err"] / plain["Z_err"] < 1.25


def test_integrate_uniform_counts_evaluations(oracle_lib):
    lat = oracle.lattice(3, 2, antithetic=1)
    res = oracle.integrate_uniform(lat, 1, -1.0, 1.0, 2, 10_002)
    assert res["n_evals"] == 10_002
    assert res["sums"][:, 0].sum() == 5001


def test_pairs_have_no_split_statistics(oracle_lib):
    lat = oracle.lattice(3, 2, antithetic=1)
    with pytest.raises(ValueError):
        oracle.split_sums(lat, 1, [1], np.full((1, 6), -1.0), np.full((1, 6), 1.0), 10)
    with pytest.raises(ValueError):
        oracle.sums(oracle.lattice(3, 2, antithetic=2), 1, [1], np.full((1, 6), -1.0),
                    np.full((1, 6), 1.0), 10)
