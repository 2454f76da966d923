"""Pins of the oracle's sampler in spherical coordinates (CPU only).

A shell rho_lo <= |u| < rho_hi is sampled uniformly in its volume: direction
from normalised normals, radius by the inverse of the rho^(d-1) law; a sample
weighs exp(-S) inside the cube and 0 outside, the shell's integral is its
volume times the mean weight.  What pins it:
  * the volume formula: 2 (rho_hi - rho_lo) for d = 1, the annulus for d = 2,
    the spherical shell for d = 3, pi^10/10! for the unit ball in d = 20;
  * points: |u| inside the shell; rho^d uniform between rho_lo^d and rho_hi^d
    (Kolmogorov-Smirnov; a uniform radius, the likeliest slip, fails it);
    directions: the polar angle uniform for d = 2 and the z coordinate uniform
    on [-1, 1] for d = 3 (Archimedes), second moments 1/d for d = 20;
  * flat weights (D = 1e300: S rounds to 0, every weight is 1): a shell inside
    the cube integrates to its volume exactly; shells out to the cube's corners
    sum to the cube's volume within the error bar; a shell beyond the corners
    integrates to 0;
  * nonlinear lattices: two sites against scipy's 2-D quadrature and 3x1
    against tensor-product Gauss-Legendre (the pins of the plain sampler), and
    4x2 against the plain cartesian sampler on the same cube, within 4 sigma.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle

from test_oracle_estimator import _gauss_legendre_box


def test_shell_volumes():
    assert oracle.sph_volume(1, 0.5, 2.0) == pytest.approx(3.0, rel=1e-15)
    assert oracle.sph_volume(2, 1.0, 3.0) == pytest.approx(8 * math.pi, rel=1e-14)
    assert oracle.sph_volume(3, 1.0, 2.0) == pytest.approx(4 / 3 * math.pi * 7, rel=1e-14)
    assert oracle.sph_volume(20, 0.0, 1.0) == pytest.approx(math.pi**10 / math.factorial(10),
                                                             rel=1e-13)
    with pytest.raises(ValueError):
        oracle.sph_volume(3, 2.0, 1.0)


def _points(d, a, b, n=4000, seed=3, stream=7):
    return np.stack([oracle.sph_point(d, seed, stream, a, b, i) for i in range(n)])


@pytest.mark.parametrize("d,a,b", [(1, 0.3, 2.0), (3, 0.0, 1.5), (3, 1.0, 2.0), (20, 2.0, 4.0),
                                   (20, 0.0, 9.0)])
def test_radius_follows_the_volume_law(d, a, b):
    u = _points(d, a, b)
    rho = np.linalg.norm(u, axis=1)
    assert np.all(rho >= a * (1 - 1e-12)) and np.all(rho <= b * (1 + 1e-12))
    x = (rho**d - a**d) / (b**d - a**d)
    assert stats.kstest(x, "uniform").pvalue > 1e-3
    if d > 1 and a > 0:
        # the likeliest slip, a radius uniform in [a, b], is far off
        assert stats.kstest((rho - a) / (b - a), "uniform").pvalue < 1e-6


def test_directions_are_uniform_on_the_sphere():
    u2 = _points(2, 0.5, 1.0)
    ang = (np.arctan2(u2[:, 1], u2[:, 0]) + math.pi) / (2 * math.pi)
    assert stats.kstest(ang, "uniform").pvalue > 1e-3
    u3 = _points(3, 0.0, 2.0)
    z = u3[:, 2] / np.linalg.norm(u3, axis=1)
    assert stats.kstest((z + 1) / 2, "uniform").pvalue > 1e-3
    u20 = _points(20, 1.0, 1.5, n=8000)
    om = u20 / np.linalg.norm(u20, axis=1, keepdims=True)
    n = om.shape[0]
    assert np.all(np.abs(om.mean(0)) < 5 / math.sqrt(n * 20))
    m2 = (om**2).mean(0)
    assert np.all(np.abs(m2 - 1 / 20) < 5 * math.sqrt(2 / (20 * 22)) / math.sqrt(n))
    c = (om[:, 0] * om[:, 1]).mean()
    assert abs(c) < 5 / (20 * math.sqrt(n))


FLAT = dict(D=1e300)  # S = R^2 / (2 D tau) rounds to 0: every weight is exactly 1


@pytest.mark.parametrize("nx,nt,B", [(2, 1, 1.0), (3, 1, 2.0), (4, 1, 1.5)])
def test_flat_weights_give_volumes(nx, nt, B):
    d = nx * nt
    lat = oracle.lattice(nx, nt, **FLAT)
    n = 20000
    # inside the inscribed ball every point is in the cube: the volume exactly
    s = oracle.sph_sums(lat, 1, B, [1], [0.2 * B], [B], [n])
    assert s[0, 1] == n and s[0, 2] == n
    res = oracle.sph_finalize(nx, d, [0.2 * B], [B], s)
    assert res["Z"] == pytest.approx(oracle.sph_volume(d, 0.2 * B, B), rel=1e-14)
    # shells out to the corners sum to the cube's volume
    edges = np.linspace(0.0, B * math.sqrt(d), 9)
    ids = np.arange(1, 9, dtype=np.uint64)
    s = oracle.sph_sums(lat, 2, B, ids, edges[:-1], edges[1:], n)
    res = oracle.sph_finalize(nx, d, edges[:-1], edges[1:], s)
    assert abs(res["Z"] - (2 * B) ** d) < 4 * res["Z_err"]
    assert res["Z_err"] < 0.02 * (2 * B) ** d
    # beyond the corners nothing is inside
    out = oracle.sph_sums(lat, 1, B, [9], [B * math.sqrt(d) * 1.01], [B * math.sqrt(d) * 2], [1000])
    assert out[0, 1] == 0.0


def _shells(d, B, k):
    edges = np.linspace(0.0, B * math.sqrt(d), k + 1)
    return np.arange(1, k + 1, dtype=np.uint64), edges[:-1], edges[1:]


def test_two_sites_against_scipy():
    B = 4.0
    kappa = 4.0
    f = lambda u1, u0, h: h(u0, u1) * math.exp(-kappa * (u1 - u0) ** 2)  # noqa: E731
    q = [integrate.dblquad(lambda u1, u0: f(u1, u0, h), -B, B, -B, B, epsabs=1e-12,
                           epsrel=1e-12)[0]
         for h in (lambda a, b: 1.0, lambda a, b: a * a, lambda a, b: a * b)]
    ids, lo, hi = _shells(2, B, 16)
    lat = oracle.lattice(2, 1)
    s = oracle.sph_sums(lat, 1, B, ids, lo, hi, 1 << 16)
    res = oracle.sph_finalize(2, 2, lo, hi, s)
    assert abs(res["Z"] - q[0]) < 4 * res["Z_err"]
    assert abs(res["C"][0] - q[1] / q[0]) < 4 * res["C_err"][0]
    assert abs(res["C"][1] - q[2] / q[0]) < 4 * res["C_err"][1]
    assert res["Z_err"] < 0.01 * q[0]


def test_nonlinear_3x1_against_quadrature():
    lat = oracle.lattice(3, 1)
    B = 2.0
    Zq, Cq = _gauss_legendre_box(lat, B, 8)
    ids, lo, hi = _shells(3, B, 16)
    s = oracle.sph_sums(lat, 5, B, ids, lo, hi, 1 << 15)
    res = oracle.sph_finalize(3, 3, lo, hi, s)
    assert abs(res["Z"] - Zq) < 4 * res["Z_err"]
    for r in range(3):
        assert abs(res["C"][r] - Cq[r]) < 4 * res["C_err"][r]
    assert res["Z_err"] < 0.01 * Zq


def test_agrees_with_the_cartesian_sampler():
    lat = oracle.lattice(4, 2)
    B = 1.0
    plain = oracle.integrate_uniform(lat, 1, -B, B, 4, 1 << 19)
    ids, lo, hi = _shells(8, B, 12)
    res = oracle.sph_finalize(4, 8, lo, hi, oracle.sph_sums(lat, 2, B, ids, lo, hi, 1 << 15))
    z = abs(res["Z"] - plain["Z"]) / math.hypot(res["Z_err"], plain["Z_err"])
    assert z < 4
    for r in range(4):
        zr = abs(res["C"][r] - plain["C"][r]) / math.hypot(res["C_err"][r], plain["C_err"][r])
        assert zr < 4, r


def test_invalid_arguments():
    lat = oracle.lattice(2, 1)
    with pytest.raises(ValueError):
        oracle.sph_sums(lat, 1, 0.0, [1], [0.0], [1.0], [10])
    with pytest.raises(ValueError):
        oracle.sph_point(3, 1, 1, 1.0, 1.0, 0)
    with pytest.raises(ValueError):
        oracle.sph_sums(oracle.lattice(2, 1, antithetic=1), 1, 1.0, [1], [0.0], [1.0], [10])
