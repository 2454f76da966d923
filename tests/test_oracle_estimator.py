"""Pins for the oracle's Monte Carlo estimator: per-subvolume sums, the plan,
the split statistics and finalize (Z, C(r) = N(r)/Z and error bars).

  * The N-sphere integrand of the paper's section 3 (Listings 1 and 2) fixes the
    error-bar convention: abserr = V s / sqrt(n) reproduces the printed 4.355e-4
    for 1e7 samples over [-1,1]^2, and the results sit within 4 sigma of the
    closed-form half-ball volumes pi^(n/2) / Gamma(n/2 + 1) / 2.
  * With the weights forced to 1 (D -> infinity) Z is the box volume exactly and
    C(r) are moments of the uniform distribution: C(0) = B^2/3, C(r > 0) = 0,
    with sigma_C(0) = B^2 sqrt(4/45)/sqrt(n).
  * Two sites and one time slice (Gaussian, exact in the box) against scipy's
    adaptive 2-D quadrature.
  * The regulated Gaussian case against the inverse of the quadratic form.
  * Tiny nonlinear lattices against tensor-product Gauss-Legendre quadrature.
  * The symmetry C(r) = C(nx - r) of the symmetric box.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = json.load(open(os.path.join(HERE, "golden", "paper_listings.json")))


def half_ball(n):
    return math.pi ** (n / 2) / math.gamma(n / 2 + 1) / 2


@pytest.mark.slow
def test_nsphere_listing2_error_convention(oracle_lib):
    g = GOLDEN["listing2"]
    r = oracle.nsphere(g["dim"], seed=1, lo=g["lo"], hi=g["hi"], n=g["samples"])
    exact = half_ball(g["dim"] + 1)
    assert abs(r["result"] - exact) < 4 * r["abserr"]
    # the paper's printed error bar for the same n and box: V s / sqrt(n)
    assert r["abserr"] == pytest.approx(g["abserr"], rel=3e-3)
    # and the paper's printed result is itself within 4 of its sigma of the truth
    assert abs(g["result"] - exact) < 4 * g["abserr"]


@pytest.mark.parametrize("dim", [1, 3, 4])
def test_nsphere_closed_forms(oracle_lib, dim):
    r = oracle.nsphere(dim, seed=2, lo=-1.0, hi=1.0, n=400_000)
    assert abs(r["result"] - half_ball(dim + 1)) < 4 * r["abserr"]
    if dim == 3:
        g = GOLDEN["listing1"]
        assert abs(g["result"] - half_ball(4)) < 4 * g["abserr"]


def test_sums_record_bruteforce(oracle_lib):
    """The record is [n, sum w, sum w^2, sum p_r w, sum (p_r w)^2, sum p_r w^2] with
    p_r = u_{0,0} u_{0,r} (first time slice, sites 0 and r)."""
    lat = oracle.lattice(4, 2, nu=0.7)
    sv = workloads.uniform_partition(8, 2.0, 2, per_sub=200, offset=17)
    got = oracle.sums(lat, 5, sv.ids, sv.lo, sv.hi, sv.n, sv.offset, nthreads=3)
    for s in range(len(sv)):
        U = oracle.points(8, 5, int(sv.ids[s]), sv.lo[s], sv.hi[s], range(17, 217))
        w = np.exp(-oracle.action_batch(lat, U))
        p = U[:, [0]] * U[:, 0:4]
        want = np.concatenate([[200, w.sum(), (w * w).sum()], (p * w[:, None]).sum(0),
                               ((p * w[:, None]) ** 2).sum(0), (p * w[:, None] ** 2).sum(0)])
        np.testing.assert_allclose(got[s], want, rtol=1e-12, atol=0)


def test_sums_independent_of_thread_count(oracle_lib):
    lat = oracle.lattice(3, 2)
    sv = workloads.random_partition(6, 2.0, 9, per_sub=300, seed=4)
    a = oracle.sums(lat, 1, sv.ids, sv.lo, sv.hi, sv.n, sv.offset, nthreads=1)
    b = oracle.sums(lat, 1, sv.ids, sv.lo, sv.hi, sv.n, sv.offset, nthreads=4)
    assert np.array_equal(a, b)


def test_split_sums_bruteforce(oracle_lib):
    lat = oracle.lattice(3, 2)
    sv = workloads.random_partition(6, 4.0, 3, per_sub=150, seed=8)
    got = oracle.split_sums(lat, 3, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    for s in range(len(sv)):
        U = oracle.points(6, 3, int(sv.ids[s]), sv.lo[s], sv.hi[s], range(150))
        w = np.exp(-oracle.action_batch(lat, U))
        mid = 0.5 * (sv.lo[s] + sv.hi[s])
        upper = U >= mid
        want = np.concatenate([(upper * w[:, None]).sum(0), (upper * (w * w)[:, None]).sum(0)])
        np.testing.assert_allclose(got[s], want, rtol=1e-12, atol=1e-300)


def test_plan_uniform_structure(oracle_lib):
    d, k = 5, 7
    ids, lo, hi = oracle.plan_uniform(d, -4.0, 4.0, k)
    assert list(ids) == list(range(2**k, 2**(k + 1)))
    vol = np.prod(hi - lo, axis=1)
    assert vol.sum() == pytest.approx(8.0**d, rel=1e-15)
    assert np.all(vol == vol[0])
    # every point of the box lies in exactly one leaf
    rng = np.random.Generator(np.random.PCG64(1))
    P = rng.uniform(-4, 4, size=(2000, d))
    inside = np.all((P[:, None, :] >= lo[None]) & (P[:, None, :] < hi[None]), axis=2)
    assert np.all(inside.sum(1) == 1)
    # level t halves dimension t mod d: dims 0, 1 bisected twice, the rest once
    widths = hi[0] - lo[0]
    assert list(widths) == [2.0, 2.0, 4.0, 4.0, 4.0]
    # the same boxes as the generic bisection of the input generator
    sv = workloads.uniform_partition(d, 4.0, k, per_sub=2)
    assert np.array_equal(sv.lo, lo) and np.array_equal(sv.hi, hi)


def test_budget_split(oracle_lib):
    n = oracle.budget_split(1000, 16)
    assert n.sum() == 1000 and n.max() - n.min() <= 1 and list(n[:8]) == [63] * 8


def test_uniform_weights_give_uniform_moments(oracle_lib):
    """D huge: S ~ 1e-30, w == 1 exactly.  Then Z = volume, sigma_Z = 0, and
    C(0) estimates E[u^2] = B^2/3 with sigma B^2 sqrt(4/45)/sqrt(n); C(r>0) -> 0."""
    B, nx, nt = 2.0, 4, 2
    lat = oracle.lattice(nx, nt, D=1e32)
    sv = workloads.uniform_partition(nx * nt, B, 3, per_sub=[5000, 7000, 3000, 4000,
                                                             6000, 2000, 8000, 5000])
    s = oracle.sums(lat, 9, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)
    assert np.array_equal(s[:, 1], s[:, 0])
    res = oracle.finalize(nx, nx * nt, sv.lo, sv.hi, s)
    assert res["Z"] == (2 * B) ** (nx * nt)
    assert res["Z_err"] == 0.0
    # stratified over 8 equal boxes with uneven n: sigma^2 = sum (1/8)^2 Var_s / n_s,
    # and each sub-box (halved in dims 0-2) keeps E[u_0^2] = B^2/3 only on average,
    # so use the reported error and the exact mean
    assert abs(res["C"][0] - B * B / 3) < 4 * res["C_err"][0]
    for r in range(1, nx):
        assert abs(res["C"][r]) < 4 * res["C_err"][r]
    # one box: the reported error equals the textbook standard error of u^2
    one = workloads.uniform_partition(nx * nt, B, 0, per_sub=40000)
    s1 = oracle.sums(lat, 10, one.ids, one.lo, one.hi, one.n, one.offset)
    r1 = oracle.finalize(nx, nx * nt, one.lo, one.hi, s1)
    assert r1["C_err"][0] == pytest.approx(B * B * math.sqrt(4 / 45) / math.sqrt(40000), rel=0.03)
    assert abs(r1["C"][0] - B * B / 3) < 4 * r1["C_err"][0]
    assert r1["ess"] == pytest.approx(40000, rel=1e-12)


def test_gaussian_two_sites_against_scipy(oracle_lib):
    """nx = 2, nt = 1: S = kappa (u1 - u0)^2 with kappa = 4 nu^2 tau / (D a^4),
    integrated over the box [-B, B]^2 by scipy's adaptive quadrature."""
    from scipy import integrate
    B, nu = 4.0, 1.0
    kappa = 4 * nu**2
    f = lambda u1, u0, h: h(u0, u1) * math.exp(-kappa * (u1 - u0) ** 2)
    Z = integrate.dblquad(lambda u1, u0: f(u1, u0, lambda a, b: 1.0), -B, B, -B, B,
                          epsabs=1e-12, epsrel=1e-12)[0]
    N0 = integrate.dblquad(lambda u1, u0: f(u1, u0, lambda a, b: a * a), -B, B, -B, B,
                           epsabs=1e-12, epsrel=1e-12)[0]
    N1 = integrate.dblquad(lambda u1, u0: f(u1, u0, lambda a, b: a * b), -B, B, -B, B,
                           epsabs=1e-12, epsrel=1e-12)[0]
    res = oracle.integrate_uniform(oracle.lattice(2, 1, nu=nu), 1, -B, B, 4, 1 << 20)
    assert abs(res["Z"] - Z) < 4 * res["Z_err"]
    assert abs(res["C"][0] - N0 / Z) < 4 * res["C_err"][0]
    assert abs(res["C"][1] - N1 / Z) < 4 * res["C_err"][1]
    assert res["Z_err"] < 2e-3 * Z


def test_regulated_gaussian_inverts_quadratic_form(oracle_lib):
    """g = 0, m2 = 1: exp(-u.Pu/2) over a box much wider than the Gaussian, so
    <u_0 u_r> = (P^-1)_{0r} (box truncation below 1e-6)."""
    nx, nt, nu, m2 = 2, 2, 0.5, 1.0
    It, Ix = np.eye(nt), np.eye(nx)
    sh = lambda n: np.roll(np.eye(n), 1, axis=1)
    Tt, Sx = np.kron(sh(nt), Ix), np.kron(It, sh(nx))
    A = (Tt - np.eye(4)) - nu * (Sx + Sx.T - 2 * np.eye(4))
    P = A.T @ A + m2 * np.eye(4)
    cov = np.linalg.inv(P)
    res = oracle.integrate_uniform(oracle.lattice(nx, nt, nu=nu, g=0.0, m2=m2), 3, -6.0, 6.0,
                                   4, 1 << 22)
    for r in range(nx):
        assert abs(res["C"][r] - cov[0, r]) < 4 * res["C_err"][r]
    assert res["C_err"][0] < 0.03 * cov[0, 0]
    Zexact = (2 * math.pi) ** 2 / math.sqrt(np.linalg.det(P))
    assert abs(res["Z"] - Zexact) < 4 * res["Z_err"]


def _gauss_legendre_box(lat, B, panels, order=8):
    x, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(-B, B, panels + 1)
    xs = np.concatenate([(edges[i] + edges[i + 1]) / 2 + (edges[i + 1] - edges[i]) / 2 * x
                         for i in range(panels)])
    ws = np.concatenate([(edges[i + 1] - edges[i]) / 2 * w for i in range(panels)])
    d = lat.d
    U = np.stack([g.ravel() for g in np.meshgrid(*([xs] * d), indexing="ij")], 1)
    W = np.ones(U.shape[0])
    for g in np.meshgrid(*([ws] * d), indexing="ij"):
        W *= g.ravel()
    f = W * np.exp(-oracle.action_batch(lat, U))
    Z = f.sum()
    return Z, np.array([(f * U[:, 0] * U[:, r]).sum() / Z for r in range(lat.nx)])


@pytest.mark.parametrize("nx,nt,B,nu", [(3, 1, 2.0, 1.0), (4, 1, 2.0, 1.0), (2, 2, 2.0, 0.5),
                                         (3, 1, 4.0, 0.5)])
def test_nonlinear_tiny_lattice_against_quadrature(oracle_lib, nx, nt, B, nu):
    lat = oracle.lattice(nx, nt, nu=nu)
    panels = (8, 12) if nx * nt <= 3 else (4, 6)
    Zq, Cq = _gauss_legendre_box(lat, B, panels[0])
    Zq2, Cq2 = _gauss_legendre_box(lat, B, panels[1])
    assert Zq == pytest.approx(Zq2, rel=1e-7)          # quadrature converged
    np.testing.assert_allclose(Cq, Cq2, rtol=1e-6, atol=1e-9 * Cq2[0])
    res = oracle.integrate_uniform(lat, 1, -B, B, 4, 1 << 21)
    assert abs(res["Z"] - Zq) < 4 * res["Z_err"]
    for r in range(nx):
        assert abs(res["C"][r] - Cq[r]) < 4 * res["C_err"][r]
    # symmetric box: C(r) = C(nx - r) exactly in quadrature
    for r in range(1, nx):
        assert Cq[r] == pytest.approx(Cq[nx - r], rel=1e-9, abs=1e-12 * Cq[0])


def test_reported_errors_match_replication_spread(oracle_lib):
    """The delta-method sigma_C agrees with the spread of independent seeds."""
    lat = oracle.lattice(3, 1)
    vals, errs = [], []
    for seed in range(1, 25):
        r = oracle.integrate_uniform(lat, seed, -2.0, 2.0, 2, 1 << 14)
        vals.append(r["C"][1])
        errs.append(r["C_err"][1])
    ratio = np.std(vals, ddof=1) / np.mean(errs)
    assert 0.6 < ratio < 1.5


def test_finalize_rejects_short_subvolumes(oracle_lib):
    sv = workloads.uniform_partition(2, 1.0, 1, per_sub=1)
    s = np.zeros((2, 9))
    s[:, 0] = 1
    with pytest.raises(ValueError):
        oracle.finalize(2, 2, sv.lo, sv.hi, s)


def test_sums_reject_empty_box(oracle_lib):
    sv = workloads.uniform_partition(2, 1.0, 1, per_sub=10)
    sv.hi[0, 1] = sv.lo[0, 1]
    with pytest.raises(ValueError):
        oracle.sums(oracle.lattice(2, 1), 1, sv.ids, sv.lo, sv.hi, sv.n, sv.offset)


def test_empty_subvolume_list(oracle_lib):
    lat = oracle.lattice(4, 2)
    out = oracle.sums(lat, 1, np.zeros(0, np.uint64), np.zeros((0, 8)), np.zeros((0, 8)),
                      np.zeros(0, np.uint64), np.zeros(0, np.uint64))
    assert out.shape == (0, 15)
